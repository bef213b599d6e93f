"""Split-BF16 path (matrix-core products with FP32 accumulation, FP32
partials) against the CPU FP64 oracle, through the C-ABI.

Tolerance 1e-5 relative, with the A_b rule for gradients (as for the FP32
path): |logL - logL*| <= 1e-5 |logL*| and |g_b - g*_b| <= 1e-5 A_b,
A_b = sum_s w_s |per-site term|.  Covers the 61-state codon workload (N = 256,
S = 1000, K = 4) in the launch configuration the benchmark times, other
state counts through the padding to 64 states, ragged pattern tails, tip
ambiguity (fully ambiguous and partial masks), zero-length branches, a
degenerate spectrum (Jukes-Cantor) and a non-diagonalisable Q (the
scaling-and-squaring fallback).
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of, jc_matrix, small

pytestmark = pytest.mark.gpu

TOL = 1e-5


def split_eval(w, t=None):
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        return ctx.logL_and_grad(w.t if t is None else t)


def check(w, label, branches=None, ref="linear"):
    logL, grad = split_eval(w)
    if ref == "naive":
        r = O.naive_gradient(*args_of(w), branches=branches)
    else:
        r = O.linear_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], TOL, branches=branches)
    print(label, rep, flush=True)
    assert rep["ok"], rep
    return logL, grad


def test_c4_codon_full_size(gpu):
    w = make_workload("C4")
    logL, grad = check(w, "C4 split-bf16 vs linear oracle")
    sample = [0, 255, 300, 509]
    r = O.naive_gradient(*args_of(w), branches=sample)
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], TOL, branches=sample)
    print("C4 split-bf16 vs naive oracle", rep, flush=True)
    assert rep["ok"], rep


@pytest.mark.parametrize("n_tips,n_patterns,n_cats,n_states,amb", [
    (2, 1, 1, 61, 0.0),      # one cherry, one pattern
    (3, 17, 2, 61, 0.1),     # ragged tail
    (40, 53, 3, 61, 0.05),   # several tiles and levels
    (33, 70, 4, 4, 0.1),     # 4 states padded to 64
    (25, 40, 2, 20, 0.05),   # 20 states
    (9, 30, 1, 64, 0.1),     # no padding
])
def test_small_shapes(gpu, n_tips, n_patterns, n_cats, n_states, amb):
    w = small(n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats, n_states=n_states, ambiguous=amb,
              seed=n_tips + n_states)
    check(w, f"split N={n_tips} S={n_patterns} K={n_cats} m={n_states}")


def test_partial_ambiguity_masks(gpu):
    w = small(n_tips=20, n_patterns=48, n_cats=2, n_states=61, ambiguous=0.0, seed=5)
    rng = np.random.default_rng(0)
    masks = w.tip_masks().copy()
    pick = rng.random(masks.shape) < 0.2
    extra = rng.integers(0, 61, size=pick.sum()).astype(np.uint64)
    masks[pick] |= np.left_shift(np.uint64(1), extra)
    w.masks = masks
    check(w, "split partial masks")


def test_zero_length_branches(gpu):
    w = small(n_tips=16, n_patterns=40, n_cats=2, n_states=61, seed=9, ambiguous=0.1)
    w.t = w.t.copy()
    w.t[[0, 3, 17, 20]] = 0.0
    check(w, "split zero lengths")


def test_degenerate_spectrum_jc(gpu):
    w = small(n_tips=12, n_patterns=40, n_cats=2, n_states=4, seed=4)
    w.Q = jc_matrix(4)
    check(w, "split JC")


def test_non_diagonalisable_q_uses_fallback(gpu):
    w = small(n_tips=10, n_patterns=33, n_cats=2, n_states=3, seed=6, mean_t=0.3)
    w.Q = np.array([[-1.0, 1.0, 0.0], [0.0, -1.0, 1.0], [0.0, 0.0, 0.0]])
    check(w, "split defective Q")


def test_long_branches(gpu):
    w = small(n_tips=30, n_patterns=64, n_cats=4, n_states=61, seed=11, mean_t=0.5)
    check(w, "split long branches")


def test_deterministic(gpu):
    w = make_workload("C4", n_tips=64, n_patterns=300)
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        a = ctx.logL_and_grad(w.t)
        b = ctx.logL_and_grad(w.t)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_logl_only_then_grad(gpu):
    w = make_workload("C4", n_tips=50, n_patterns=200)
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        l1, g1 = ctx.logL_and_grad(w.t)
        l2 = ctx.logL(w.t)
        g2 = ctx.grad()
    assert l1 == l2 and np.array_equal(g1, g2)


def test_server_precisions(gpu):
    # every precision serves (split-BF16 included); an unknown one is refused
    h = B.pg_server_create(0, B.PG_SPLIT_BF16, 1 << 30, 4)
    B.pg_server_destroy(h)
    with pytest.raises(B.PhyloGradError) as e:
        B.pg_server_create(0, 7, 1 << 30, 4)
    assert e.value.code == B.PG_E_UNSUPPORTED


@pytest.mark.parametrize("n_tips,n_cats,n_states", [(7, 2, 61), (20, 3, 4), (12, 4, 20)])
def test_hessian_split(gpu, n_tips, n_cats, n_states):
    """Section 2.7 on the split-BF16 path: Q^2 m split in three BF16 parts;
    within 1e-5 of the FP64 oracle with the cancellation-free scale
    sum_s w_s (|d2L_s/L_s| + (dL_s/L_s)^2)."""
    w = small(n_tips=n_tips, n_cats=n_cats, n_states=n_states, n_patterns=37, seed=60 + n_tips,
              ambiguous=0.05, mean_t=0.15)
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        logL, grad = ctx.logL_and_grad(w.t)
        g2, h = ctx.hessian_diag()
    assert np.array_equal(grad, g2)
    nh = O.naive_hessian_diag(*args_of(w))
    rel = np.abs(h - nh["hess"]) / np.maximum(nh["abs_hess"], np.finfo(float).tiny)
    print("split Hessian", n_states, "A-rule max", rel.max(), flush=True)
    assert (rel <= TOL).all(), rel.max()
