"""Partial re-evaluation (pg_logL_update): after changing a few branch
lengths, the logL and the partials left for pg_grad are bitwise those of a
full evaluation at the new lengths; agreement with the oracle; errors."""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu


def _full(w, t, precision):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        return ctx.logL_and_grad(t)


@pytest.mark.parametrize("precision", [B.PG_FP64, B.PG_FP32])
@pytest.mark.parametrize("name,kw", [("C1", dict(n_tips=40, n_patterns=53, n_cats=3, ambiguous_frac=0.1)),
                                     ("C2", dict()),
                                     ("C1", dict(n_tips=24, n_patterns=40, n_cats=2, n_states=20))])
def test_updates_equal_full_evaluation_bitwise(gpu, name, kw, precision):
    w = make_workload(name, seed=41, **kw)
    B_ = len(w.t)
    rng = np.random.default_rng(0)
    root_children = [b for b in range(B_) if w.parent[b] == 2 * w.n_tips - 2]
    steps = [[0], [B_ - 1], [w.n_tips + 1], root_children, list(rng.choice(B_, 5, replace=False)), [3, 3]]
    t = w.t.copy()
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        ctx.logL(t)
        for bs in steps:
            new = t[bs] * np.exp(rng.normal(0.0, 0.3, size=len(bs)))
            new[-1] = new[-1] if len(bs) < 2 or bs[0] != bs[-1] else new[0] * 1.1
            logL = ctx.logL_update(bs, new)
            for b, v in zip(bs, new):
                t[b] = v
            ref_l, ref_g = _full(w, t, precision)
            assert logL == ref_l, (bs, logL, ref_l)
            g = ctx.grad()
            assert np.array_equal(g, ref_g), bs
    if precision == B.PG_FP64 and name == "C1":
        w2 = make_workload(name, seed=41, **kw)
        w2.t = t
        r = O.linear_gradient(*args_of(w2))
        assert abs(logL - r["logL"]) <= 1e-10 * abs(r["logL"])


@pytest.mark.parametrize("name,kw", [("C1", dict(n_tips=30, n_patterns=45, n_cats=2, n_states=61)),
                                     ("C4", dict(n_tips=64, n_patterns=300))])
def test_split_updates_equal_full_evaluation_bitwise(gpu, name, kw):
    """Split-BF16 (codon-sized state spaces): the dirty-path update leaves
    the same bits as a full evaluation, and the updated logL and gradient
    meet the oracle at the path's tolerance (1e-5, A_b rule)."""
    w = make_workload(name, seed=43, **kw)
    B_ = len(w.t)
    rng = np.random.default_rng(3)
    root_children = [b for b in range(B_) if w.parent[b] == 2 * w.n_tips - 2]
    steps = [[1], [B_ - 1], root_children, list(rng.choice(B_, 4, replace=False))]
    t = w.t.copy()
    with B.Context(0, B.PG_SPLIT_BF16) as ctx:
        ctx.set_workload(w)
        ctx.logL(t)
        for bs in steps:
            new = t[bs] * np.exp(rng.normal(0.0, 0.3, size=len(bs)))
            logL = ctx.logL_update(bs, new)
            t[bs] = new
            ref_l, ref_g = _full(w, t, B.PG_SPLIT_BF16)
            assert logL == ref_l, (bs, logL, ref_l)
            g = ctx.grad()
            assert np.array_equal(g, ref_g), bs
    w2 = make_workload(name, seed=43, **kw)
    w2.t = t
    r = O.linear_gradient(*args_of(w2))
    rep = O.parity_report(logL, g, r["logL"], r["grad"], r["abs_grad"], 1e-5)
    print("split after updates vs oracle", name, rep, flush=True)
    assert rep["ok"], rep


def test_c2_update_against_the_oracle(gpu):
    """At the full 4-state size: logL after single-branch, root and
    multi-branch updates, and the gradient of the updated partials (pg_grad),
    against the FP64 oracle at the new lengths (1e-10, A_b rule)."""
    w = make_workload("C2")
    B_ = len(w.t)
    rng = np.random.default_rng(9)
    root_children = [b for b in range(B_) if w.parent[b] == 2 * w.n_tips - 2]
    t = w.t.copy()
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        ctx.logL(t)
        for bs in ([17], root_children, list(rng.choice(B_, 4, replace=False))):
            new = t[bs] * np.exp(rng.normal(0.0, 0.5, size=len(bs)))
            logL = ctx.logL_update(bs, new)
            t[bs] = new
        grad = ctx.grad()
    w2 = make_workload("C2")
    w2.t = t
    r = O.linear_gradient(*args_of(w2))
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], 1e-10)
    print("C2 after updates vs oracle", rep, flush=True)
    assert rep["ok"], rep


def test_update_errors(gpu):
    w = small(n_tips=10, n_patterns=20)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_update([0], [0.1])
        assert e.value.code == B.PG_E_STATE
        ctx.logL(w.t)
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_update([len(w.t)], [0.1])
        assert e.value.code == B.PG_E_INVALID
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_update([0], [-1.0])
        assert e.value.code == B.PG_E_INVALID
        ctx.logL_update([1], [0.2])
        import torch
        d_t = torch.tensor(w.t, device="cuda", dtype=torch.float64)
        d_l = torch.zeros(1, device="cuda", dtype=torch.float64)
        ctx.logL_and_grad_device(d_t.data_ptr(), d_l.data_ptr(), 0)
        torch.cuda.synchronize()
        with pytest.raises(B.PhyloGradError) as e:
            ctx.logL_update([0], [0.1])
        assert e.value.code == B.PG_E_STATE
