"""Pins of the oracle with a non-homogeneous model (one rate matrix per
branch, Section 2.1): enumeration against pruning and the enumerated
derivative against the naive and linear gradients, the homogeneous special
case, and Richardson differences."""
import numpy as np

import oracle as O
from synth.workloads import branch_models
from tests._fixtures import args_of, small


def _nonhom(n_tips, n_models, seed, n_cats=2, n_patterns=25):
    w = small(n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats, seed=seed, ambiguous=0.1, mean_t=0.2)
    Qs, model = branch_models(w, n_models, seed=seed)
    a = list(args_of(w))
    a[2] = Qs[model]          # [2N-2, m, m]
    return w, a


def test_identical_branch_matrices_equal_homogeneous():
    w = small(n_tips=9, n_patterns=30, n_cats=2, seed=3)
    a = list(args_of(w))
    hom = O.linear_gradient(*a)
    a[2] = np.broadcast_to(w.Q, (len(w.t),) + w.Q.shape).copy()
    per = O.linear_gradient(*a)
    assert per["logL"] == hom["logL"] and np.array_equal(per["grad"], hom["grad"])


def test_enumeration_equals_pruning():
    for seed in (1, 2, 3):
        _, a = _nonhom(5, 3, seed)
        brute = O.brute_site_likelihoods(*a)
        prune = O.site_log_likelihoods(*a)
        assert np.allclose(np.log(brute), prune, rtol=0, atol=1e-12)


def test_enumerated_derivative_equals_naive_and_linear():
    for seed in (4, 5):
        _, a = _nonhom(5, 3, seed)
        b_logL, b_grad, _, _ = O.brute_gradient(*a)
        nv = O.naive_gradient(*a)
        lin = O.linear_gradient(*a)
        assert abs(nv["logL"] - b_logL) <= 1e-13 * abs(b_logL)
        assert np.all(np.abs(nv["grad"] - b_grad) <= 1e-11 * nv["abs_grad"])
        assert np.all(np.abs(lin["grad"] - b_grad) <= 1e-11 * nv["abs_grad"])


def test_linear_equals_naive_larger_tree():
    _, a = _nonhom(14, 4, 7, n_cats=3, n_patterns=40)
    nv = O.naive_gradient(*a)
    lin = O.linear_gradient(*a)
    assert abs(lin["logL"] - nv["logL"]) <= 1e-12 * abs(nv["logL"])
    assert np.all(np.abs(lin["grad"] - nv["grad"]) <= 1e-11 * nv["abs_grad"])
    nh = O.naive_hessian_diag(*a)
    assert np.all(np.abs(lin["hess"] - nh["hess"]) <= 1e-10 * nh["abs_hess"])


def test_richardson_differences():
    _, a = _nonhom(8, 3, 9)
    lin = O.linear_gradient(*a)
    t = a[1]
    for b in (0, 5, len(t) - 1):
        def f(h, b=b):
            tt = t.copy()
            tt[b] += h
            aa = list(a)
            aa[1] = tt
            return O.log_likelihood(*aa)
        d = O.richardson_directional(f, 1e-3)
        assert abs(d - lin["grad"][b]) <= 1e-7 * max(1.0, abs(lin["grad"][b]))


def test_branch_matrix_matters():
    w, a = _nonhom(8, 3, 11)
    base = O.log_likelihood(*a)
    a2 = list(a)
    Q2 = a[2].copy()
    Q2[3] = Q2[3] * 2.0
    a2[2] = Q2
    assert abs(O.log_likelihood(*a2) - base) > 1e-6
