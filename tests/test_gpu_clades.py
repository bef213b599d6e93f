"""Depth-first clade walks of the small-state traversals (subtrees of at
most 32 internal nodes walked by one node slot, the nodes above them walked
level by level), against the CPU FP64 oracle through the C-ABI.

The C2-sized cases in test_gpu_parity already run through clades; these
cover the shapes that stress the planner and the kernels' corner paths:
a tree whose schedule is too large to stage in LDS (read from memory), a
caterpillar (one small clade, a long level-by-level chain above it), a
tree that is a single clade below the root, ambiguous tips inside clades,
FP32, the Hessian diagonal, and partial re-evaluation on a clade tree.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu

TOL = {B.PG_FP64: 1e-10, B.PG_FP32: 1e-5}


def caterpillar(n):
    """Internal node n + i joins tip i + 1 and node n + i - 1 (tips 0, 1 at
    the bottom); the root is 2n - 2."""
    par = np.full(2 * n - 1, -1, np.int32)
    par[0] = par[1] = n
    for i in range(1, n - 1):
        par[i + 1] = n + i
        par[n + i - 1] = n + i
    return par


def check(w, precision, label):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        logL, grad = ctx.logL_and_grad(w.t)
    r = O.linear_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], TOL[precision])
    print(label, rep, flush=True)
    assert rep["ok"], rep


@pytest.mark.parametrize("precision", [B.PG_FP64, B.PG_FP32])
@pytest.mark.parametrize("n_cats,n_patterns", [(3, 53), (5, 17), (1, 33), (2, 200)])
def test_clade_launch_tile_groups(gpu, precision, n_cats, n_patterns):
    # the separate clade launches give a wavefront four tiles in
    # pattern-block-major order: groups that mix categories and pattern
    # blocks, and a short last group (53 patterns x 3 categories: 12 tiles;
    # 17 x 5: 10 tiles; 33 x 1: 3 tiles; 200 x 2: 26 tiles)
    w = make_workload("C2", n_tips=120, n_patterns=n_patterns, n_cats=n_cats)
    check(w, precision, f"N=120 S={n_patterns} K={n_cats} precision={precision}")


@pytest.mark.parametrize("precision", [B.PG_FP64, B.PG_FP32])
def test_schedule_in_memory(gpu, precision):
    # 3000 tips: 2999 schedule entries exceed the LDS budget for staging
    w = make_workload("C2", n_tips=3000, n_patterns=37)
    check(w, precision, f"N=3000 S=37 precision={precision}")


@pytest.mark.parametrize("precision", [B.PG_FP64, B.PG_FP32])
def test_caterpillar(gpu, precision):
    w = small(n_tips=300, n_patterns=45, n_cats=2, ambiguous=0.1, seed=7)
    w.parent = caterpillar(300)
    check(w, precision, f"caterpillar N=300 precision={precision}")


def test_single_clade_below_root(gpu):
    # 30 tips: both subtrees of the root are clades, the top is the root
    w = small(n_tips=30, n_patterns=50, n_cats=3, ambiguous=0.2, seed=3)
    check(w, B.PG_FP64, "N=30 two clades")


def test_ambiguous_tips_in_clades(gpu):
    w = make_workload("C2", n_tips=400, n_patterns=40)
    rng = np.random.default_rng(5)
    masks = w.tip_masks().copy()
    full = np.uint64(15)
    pick = rng.random(masks.shape)
    masks[pick < 0.05] = full                                   # gaps
    extra = rng.integers(0, 4, size=masks.shape).astype(np.uint64)
    part = pick > 0.97
    masks[part] |= np.left_shift(np.uint64(1), extra[part])     # partial ambiguity
    w.masks = masks
    check(w, B.PG_FP64, "N=400 ambiguous tips")


def test_hessian_on_clade_tree(gpu):
    w = make_workload("C2", n_tips=200, n_patterns=30)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        ctx.logL(w.t)
        g, h = ctx.hessian_diag()
    r = O.linear_gradient(*args_of(w))
    assert np.all(np.abs(g - r["grad"]) <= 1e-10 * r["abs_grad"])
    assert np.all(np.abs(h - r["hess"]) <= 1e-10 * r["abs_hess"])


def test_update_on_clade_tree(gpu):
    # partial re-evaluation walks the changed paths level by level over
    # messages the clade walk wrote; bitwise equal to a full evaluation
    w = make_workload("C2", n_tips=300, n_patterns=40)
    t = w.t.copy()
    rng = np.random.default_rng(2)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        ctx.logL(t)
        for bs in ([5], [400, 17], list(rng.choice(len(t), 6, replace=False))):
            new = t[bs] * 1.3
            l = ctx.logL_update(bs, new)
            t[bs] = new
            with B.Context(0, B.PG_FP64) as c2:
                c2.set_workload(w)
                assert c2.logL(t) == l
