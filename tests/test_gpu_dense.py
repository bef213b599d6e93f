"""The dense-state (20 amino-acid) path on the matrix cores, against the oracle.

FP64 and FP32 partials with every product of P, P^T, Q and Q^2 as 16 x 16 x 4
MFMAs: logL and all branch gradients within 1e-10 (FP64) or 1e-5 (FP32) of
the FP64 oracle with the A_b rule (Sections 2.3-2.6), on ragged shapes (a
single cherry, a 17-pattern tail), partial and full ambiguity, zero-length
branches, the full 20-state workload N=500, S=3000, K=4, the Hessian
diagonal (Section 2.7), and bitwise repeatability.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_12146_amd import binding as B
from synth import make_workload
from tests._fixtures import args_of, small

pytestmark = pytest.mark.gpu

TOL = {B.PG_FP64: 1e-10, B.PG_FP32: 1e-5}


def gpu_eval(w, precision):
    with B.Context(0, precision) as ctx:
        ctx.set_workload(w)
        return ctx.logL_and_grad(w.t)


def check(w, precision, ref=None, branches=None):
    logL, grad = gpu_eval(w, precision)
    r = ref if ref is not None else O.naive_gradient(*args_of(w))
    rep = O.parity_report(logL, grad, r["logL"], r["grad"], r["abs_grad"], TOL[precision], branches=branches)
    print("m", w.n_states, precision, w.n_tips, w.n_patterns, w.n_cats, rep, flush=True)
    assert rep["ok"], rep
    return logL, grad


@pytest.mark.parametrize("precision", [B.PG_FP64, B.PG_FP32])
@pytest.mark.parametrize("n_tips,n_patterns,n_cats,amb", [
    (2, 1, 1, 0.0),       # one cherry, one pattern
    (3, 17, 2, 0.1),      # ragged tail: 17 patterns -> 2 tiles
    (37, 53, 3, 0.1),     # several tiles and levels
    (90, 40, 4, 0.02),
])
def test_small_shapes(gpu, precision, n_tips, n_patterns, n_cats, amb):
    w = small(n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats, n_states=20, ambiguous=amb,
              seed=40 + n_tips, mean_t=0.1)
    check(w, precision)


def test_partial_ambiguity_and_zero_lengths(gpu):
    w = small(n_tips=20, n_patterns=48, n_cats=2, n_states=20, ambiguous=0.05, seed=5)
    rng = np.random.default_rng(1)
    masks = w.tip_masks().copy()
    pick = rng.random(masks.shape) < 0.15
    sets = np.array([(1 << a) | (1 << b) | (1 << c) for a, b, c in rng.integers(0, 20, size=(30, 3))],
                    dtype=np.uint64)
    masks[pick] = rng.choice(sets, size=pick.sum())
    w.masks = masks
    w.t = w.t.copy()
    w.t[[0, 7, 21, 30]] = 0.0
    for precision in (B.PG_FP64, B.PG_FP32):
        check(w, precision)


@pytest.fixture(scope="module")
def c5():
    w = make_workload("C5")
    return w, O.linear_gradient(*args_of(w))


def test_c5_fp64_all_branches(gpu, c5):
    w, ref = c5
    logL, grad = check(w, B.PG_FP64, ref)
    sample = [0, 1, 250, 500, 997]
    nv = O.naive_gradient(*args_of(w), branches=sample)
    rep = O.parity_report(logL, grad, nv["logL"], nv["grad"], nv["abs_grad"], 1e-10, branches=sample)
    assert rep["ok"], rep


def test_c5_fp32_all_branches(gpu, c5):
    w, ref = c5
    check(w, B.PG_FP32, ref)


def test_repeatable_bitwise(gpu):
    w = small(n_tips=60, n_patterns=70, n_cats=4, n_states=20, seed=8)
    with B.Context(0, B.PG_FP64) as ctx:
        ctx.set_workload(w)
        a = ctx.logL_and_grad(w.t)
        b = ctx.logL_and_grad(w.t)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_hessian_fp32(gpu):
    w = small(n_tips=15, n_cats=2, n_states=20, n_patterns=37, seed=19, ambiguous=0.05, mean_t=0.15)
    with B.Context(0, B.PG_FP32) as ctx:
        ctx.set_workload(w)
        ctx.logL_and_grad(w.t)
        g2, h = ctx.hessian_diag()
    nh = O.naive_hessian_diag(*args_of(w))
    rel = np.abs(h - nh["hess"]) / np.maximum(nh["abs_hess"], np.finfo(float).tiny)
    print("dense FP32 Hessian, A rule max", rel.max(), flush=True)
    assert (rel <= 1e-5).all()


def _chain_q(m):
    """A defective generator (one Jordan block): x -> x + 1 at rate 1, the
    last state absorbing.  No eigen-decomposition exists, so the transition
    matrices come from scaling and squaring."""
    Q = np.zeros((m, m))
    for x in range(m - 1):
        Q[x, x] = -1.0
        Q[x, x + 1] = 1.0
    return Q


def _cyclic_q(m):
    """x -> x + 1 (mod m) at rate 1: eigenvalues e^{2 pi i k / m} - 1, so the
    decomposition has conjugate pairs (the 2 x 2 blocks of the real form)."""
    Q = -np.eye(m)
    for x in range(m):
        Q[x, (x + 1) % m] = 1.0
    return Q


@pytest.mark.parametrize("m", [4, 20])
def test_eigen_route_and_its_fallbacks(gpu, m):
    """Transition matrices for a random Q, a cyclic Q with conjugate pairs,
    Jukes-Cantor with an (m-1)-fold eigenvalue and a defective Q, each
    against the oracle (which uses SciPy's expm), FP64 and FP32.  The
    20-state kernels take the eigen-decomposition for the first three and
    scaling and squaring for the defective one; the 4-state kernels always
    use scaling and squaring."""
    from tests._fixtures import jc_matrix
    from synth.workloads import simulate_sites
    cases = (("random", None), ("cyclic", _cyclic_q(m)), ("jukes-cantor", jc_matrix(m)),
             ("defective", _chain_q(m)))
    for label, Q in cases:
        w = small(n_tips=25, n_patterns=40, n_cats=2, n_states=m, seed=71, ambiguous=0.05, mean_t=0.2)
        if Q is not None:
            w.Q = Q
        if label in ("defective", "cyclic"):
            # uniform tips can need a jump over most of the chain on one short
            # branch, which the truncated series prices at exactly zero; tips
            # simulated under the chain itself keep every pattern likely
            rng = np.random.Generator(np.random.PCG64(72))
            w.tip_states = simulate_sites(w.parent, w.t, Q, w.pi, w.rates, w.cat_weights, 40, rng)
        V, Vinv, re, im, kind, cond, resid = B.pg_eigensystem(w.Q) if label != "defective" else (None,) * 7
        print("eigen route", m, label, cond, resid, None if kind is None else list(kind), flush=True)
        if label == "cyclic":
            assert (np.asarray(kind) != 0).any()
        for precision in (B.PG_FP64, B.PG_FP32):
            check(w, precision)
