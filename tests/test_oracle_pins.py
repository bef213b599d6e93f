"""Pins of the CPU oracle against facts it does not compute itself.

Each test fixes one part of the oracle to something outside it: a closed
form, brute-force enumeration of Eq. (likelihood), an invariant of the
model (probabilities sum to one, Eq. forwardBackwardLikelihood at every
node, the pulley principle), or finite differences.  A plausible slip in the
oracle (a dropped term, P where P^T belongs, a wrong sign or index) fails
at least one of them.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from oracle.fd import richardson_directional
from oracle.transition import transition_derivatives, transition_matrices
from synth import make_workload, random_rate_matrix, states_to_masks
from tests._fixtures import all_patterns, args_of, gtr_matrix, jc_matrix, small

# ---------------------------------------------------------------- transition matrices


def test_transition_rows_semigroup_and_derivative():
    rng = np.random.default_rng(1)
    Q = random_rate_matrix(4, rng)
    rates = np.array([0.3, 1.7])
    t = np.array([0.0, 0.01, 0.4, 2.5])
    P = transition_matrices(Q, rates, t)
    assert np.abs(P.sum(axis=3) - 1).max() < 1e-14
    assert P.min() > -1e-15
    assert np.abs(P[0] - np.eye(4)).max() == 0.0          # t = 0 gives the identity
    # semigroup: P(s) P(u) = P(s + u)
    Ps = transition_matrices(Q, [1.0], [0.3])[0, 0]
    Pu = transition_matrices(Q, [1.0], [0.45])[0, 0]
    Psu = transition_matrices(Q, [1.0], [0.75])[0, 0]
    assert np.abs(Ps @ Pu - Psu).max() < 1e-14
    # dP/dt = gamma Q P, against a Richardson difference of the matrix function
    D = transition_derivatives(Q, rates, P)
    for b in range(1, 4):
        for l in range(2):
            num = np.array([[richardson_directional(
                lambda h, x=x, y=y: transition_matrices(Q, [rates[l]], [t[b] + h])[0, 0][x, y],
                h=min(1e-2, t[b] / 2)) for y in range(4)] for x in range(4)])
            assert np.abs(num - D[b, l]).max() < 1e-9
    # Q P = P Q (used to move Q through P in the gradient)
    assert np.abs(Q @ P[2, 1] - P[2, 1] @ Q).max() < 1e-14


def test_transition_jc69_closed_form():
    Q = jc_matrix(4)
    for t in (0.0, 0.05, 0.7, 3.0):
        P = transition_matrices(Q, [1.0], [t])[0, 0]
        same = 0.25 + 0.75 * np.exp(-4.0 * t / 3.0)
        diff = 0.25 - 0.25 * np.exp(-4.0 * t / 3.0)
        assert np.abs(np.diag(P) - same).max() < 1e-15
        off = P[~np.eye(4, dtype=bool)]
        assert np.abs(off - diff).max() < 1e-15


# ---------------------------------------------------------------- likelihood


@pytest.mark.parametrize("n_tips,n_cats,amb", [(2, 1, 0.0), (3, 1, 0.2), (4, 2, 0.1), (5, 3, 0.1),
                                                (6, 1, 0.05)])
def test_pruning_equals_enumeration(n_tips, n_cats, amb):
    w = small(n_tips=n_tips, n_cats=n_cats, ambiguous=amb, n_patterns=25, seed=n_tips * 11)
    Lb = O.brute_site_likelihoods(*args_of(w))
    ll = O.site_log_likelihoods(*args_of(w))
    assert np.abs(ll - np.log(Lb)).max() < 1e-13
    assert abs(O.log_likelihood(*args_of(w)) - np.sum(w.weights * np.log(Lb))) < 1e-12 * abs(
        np.sum(w.weights * np.log(Lb)))


@pytest.mark.parametrize("n_tips,m", [(2, 4), (3, 4), (5, 4), (3, 5)])
def test_likelihood_sums_to_one_over_all_patterns(n_tips, m):
    rng = np.random.default_rng(n_tips * m)
    w = small(n_tips=n_tips, n_states=m, n_cats=2, seed=n_tips + m)
    masks = all_patterns(n_tips, m)
    weights = np.ones(masks.shape[1])
    ll = O.site_log_likelihoods(w.parent, w.t, w.Q, w.pi, w.rates, w.cat_weights, masks, weights)
    assert abs(np.exp(ll).sum() - 1.0) < 1e-13
    del rng


def test_fully_ambiguous_site_has_likelihood_one_and_zero_gradient():
    w = small(n_tips=7, n_cats=2, n_patterns=6, seed=3)
    masks = w.tip_masks().copy()
    masks[:, 2] = np.uint64(0xF)
    ll = O.site_log_likelihoods(*args_of(w)[:6], masks, w.weights)
    assert abs(ll[2]) < 1e-14
    nv = O.naive_gradient(*args_of(w)[:6], masks, w.weights)
    assert np.abs(nv["site_terms"][:, 2]).max() < 1e-13


def test_jc69_two_taxon_closed_form():
    Q = jc_matrix(4)
    pi = np.full(4, 0.25)
    parent = np.array([2, 2, -1])
    t = np.array([0.13, 0.41])
    masks = states_to_masks(np.array([[0, 0, 2], [0, 1, 2]], dtype=np.int16), 4)
    weights = np.array([2.0, 3.0, 1.0])
    e = np.exp(-4.0 * t.sum() / 3.0)
    L_same = 0.25 * (0.25 + 0.75 * e)
    L_diff = 0.25 * (0.25 - 0.25 * e)
    expect = 2 * np.log(L_same) + 3 * np.log(L_diff) + np.log(L_same)
    got = O.log_likelihood(parent, t, Q, pi, [1.0], [1.0], masks, weights)
    assert abs(got - expect) < 1e-14 * abs(expect)
    # d/dt_1 in closed form (either branch: JC is reversible and stationary)
    dsame = 0.25 * 0.75 * (-4.0 / 3.0) * e / L_same
    ddiff = 0.25 * (-0.25) * (-4.0 / 3.0) * e / L_diff
    g_expect = 3 * dsame + 3 * ddiff
    nv = O.naive_gradient(parent, t, Q, pi, [1.0], [1.0], masks, weights)
    assert np.abs(nv["grad"] - g_expect).max() < 1e-13 * abs(g_expect)


def test_pulley_principle_reversible_stationary():
    rng = np.random.default_rng(5)
    Q, pi = gtr_matrix(rng)
    w = small(n_tips=6, n_cats=2, seed=9)
    root = len(w.parent) - 1
    kids = np.nonzero(w.parent == root)[0]
    a, b = kids
    t2 = w.t.copy()
    shift = 0.4 * t2[a]
    t2[a] -= shift
    t2[b] += shift
    l1 = O.log_likelihood(w.parent, w.t, Q, pi, w.rates, w.cat_weights, w.tip_masks(), w.weights)
    l2 = O.log_likelihood(w.parent, t2, Q, pi, w.rates, w.cat_weights, w.tip_masks(), w.weights)
    assert abs(l1 - l2) < 1e-12 * abs(l1)
    nv = O.naive_gradient(w.parent, w.t, Q, pi, w.rates, w.cat_weights, w.tip_masks(), w.weights)
    assert abs(nv["grad"][a] - nv["grad"][b]) < 1e-11 * nv["abs_grad"][a]


def test_non_reversible_root_branches_differ():
    """The pulley identity must fail for a non-reversible, non-stationary model."""
    w = small(n_tips=6, n_cats=2, seed=9)
    root = len(w.parent) - 1
    a, b = np.nonzero(w.parent == root)[0]
    nv = O.naive_gradient(*args_of(w))
    assert abs(nv["grad"][a] - nv["grad"][b]) > 1e-3 * nv["abs_grad"][a]


def test_rescaled_equals_unscaled_and_single_category_reduction():
    w = small(n_tips=12, n_cats=4, n_patterns=30, seed=4)
    a = O.site_log_likelihoods(*args_of(w), rescale=True)
    b = O.site_log_likelihoods(*args_of(w), rescale=False)
    assert np.abs(a - b).max() < 1e-12
    # all categories at rate 1 is the one-category model
    ones = np.ones(4)
    c = O.site_log_likelihoods(w.parent, w.t, w.Q, w.pi, ones, w.cat_weights, w.tip_masks(),
                               w.weights)
    d = O.site_log_likelihoods(w.parent, w.t, w.Q, w.pi, [1.0], [1.0], w.tip_masks(), w.weights)
    assert np.abs(c - d).max() < 1e-13


def test_rescaling_keeps_large_trees_finite():
    w = make_workload("C2", n_tips=300, n_patterns=50)
    ll = O.site_log_likelihoods(*args_of(w))
    assert np.isfinite(ll).all()
    lu = O.site_log_likelihoods(*args_of(w), rescale=False)
    # 300 tips underflow-free here, so both routes agree
    assert np.abs(ll - lu).max() < 1e-10 * np.abs(ll).max()


# ---------------------------------------------------------------- gradient


@pytest.mark.parametrize("n_tips,m,n_cats", [(2, 4, 1), (4, 4, 2), (6, 4, 1), (6, 4, 3),
                                               (3, 20, 2), (4, 20, 1), (3, 61, 1)])
def test_naive_gradient_equals_enumerated_derivative(n_tips, m, n_cats):
    w = small(n_tips=n_tips, n_states=m, n_cats=n_cats, n_patterns=12 if m > 4 else 30,
              seed=100 + n_tips + m)
    if m == 61:
        w.Q = make_workload("C4", n_tips=4, n_patterns=2).Q
        w.pi = make_workload("C4", n_tips=4, n_patterns=2).pi
        w.tip_states = np.random.default_rng(3).integers(0, 61, size=w.tip_states.shape).astype(
            np.int16)
    lb, gb, _, _ = O.brute_gradient(*args_of(w))
    nv = O.naive_gradient(*args_of(w))
    assert abs(nv["logL"] - lb) < 1e-13 * abs(lb)
    assert (np.abs(nv["grad"] - gb) <= 1e-12 * nv["abs_grad"]).all()


def test_linear_pre_order_gradient_equals_naive():
    w = make_workload("C2", n_tips=60, n_patterns=80)
    nv = O.naive_gradient(*args_of(w))
    lin = O.linear_gradient(*args_of(w))
    assert abs(lin["logL"] - nv["logL"]) < 1e-13 * abs(nv["logL"])
    assert (np.abs(lin["grad"] - nv["grad"]) <= 1e-12 * nv["abs_grad"]).all()


def test_forward_backward_identity_at_every_node():
    """q_k^T p_k is the same site likelihood at every node."""
    w = small(n_tips=9, n_cats=3, n_patterns=20, seed=12)
    p, lsp, q, lsq = O.linear_partials(*args_of(w))
    ll = O.site_log_likelihoods(*args_of(w))
    for k in p:
        val = np.einsum("l,lsx,lsx->s", w.cat_weights, p[k], q[k])
        assert np.abs(np.log(val) + lsp[k] + lsq[k] - ll).max() < 1e-12


def test_pre_order_vector_sums_to_likelihood_with_subtree_masked():
    """sum_x q_i(x) = P(data with every tip below i fully ambiguous)."""
    w = small(n_tips=8, n_cats=2, n_patterns=15, seed=21)
    p, lsp, q, lsq = O.linear_partials(*args_of(w))
    parent = w.parent
    n = w.n_tips
    for i in (3, n + 1, n + 3):
        below = [v for v in range(n) if _is_below(parent, v, i)]
        masks = w.tip_masks().copy()
        masks[below] = np.uint64(0xF)
        ll = O.site_log_likelihoods(*args_of(w)[:6], masks, w.weights)
        lhs = np.log(np.einsum("l,lsx->s", w.cat_weights, q[i])) + lsq[i]
        assert np.abs(lhs - ll).max() < 1e-12


def _is_below(parent, v, i):
    while v != -1:
        if v == i:
            return True
        v = parent[v]
    return False


def test_euler_identity_for_the_length_scaling_direction():
    """sum_b t_b g_b = d/dc logL(c t) at c = 1."""
    w = small(n_tips=10, n_cats=4, n_patterns=40, seed=2)
    nv = O.naive_gradient(*args_of(w))
    f = lambda h: O.log_likelihood(w.parent, w.t * (1 + h), *args_of(w)[2:])
    d = richardson_directional(f, h=1e-3)
    lhs = float(np.dot(w.t, nv["grad"]))
    assert abs(lhs - d) < 1e-9 * np.dot(w.t, nv["abs_grad"])


def test_central_fd_agrees_loosely():
    w = small(n_tips=7, n_cats=2, n_patterns=30, seed=8, mean_t=0.2)
    nv = O.naive_gradient(*args_of(w))
    fd = O.central_fd_gradient(*args_of(w), h=1e-6)
    assert (np.abs(fd - nv["grad"]) <= 1e-3 + 1e-4 * np.abs(nv["grad"])).all()


def test_gradient_vanishes_on_very_long_branch():
    w = small(n_tips=6, n_cats=1, n_patterns=30, seed=31)
    t = w.t.copy()
    t[2] = 200.0
    nv = O.naive_gradient(w.parent, t, *args_of(w)[2:])
    assert abs(nv["grad"][2]) < 1e-12 * max(1.0, nv["abs_grad"][np.isfinite(nv["abs_grad"])].max())


def test_zero_length_branch_is_allowed():
    w = small(n_tips=6, n_cats=2, seed=17)
    t = w.t.copy()
    t[[1, 7]] = 0.0
    lb, gb, _, _ = O.brute_gradient(w.parent, t, *args_of(w)[2:])
    nv = O.naive_gradient(w.parent, t, *args_of(w)[2:])
    assert (np.abs(nv["grad"] - gb) <= 1e-12 * nv["abs_grad"]).all()


# ---------------------------------------------------------------- Hessian diagonal


def test_hessian_diag_naive_linear_and_fd():
    w = small(n_tips=7, n_cats=3, n_patterns=25, seed=41, mean_t=0.2)
    nh = O.naive_hessian_diag(*args_of(w))
    lin = O.linear_gradient(*args_of(w))
    assert (np.abs(nh["hess"] - lin["hess"]) <= 1e-11 * nh["abs_hess"]).all()
    # derivative of the (enumerated) gradient by Richardson differences
    for b in (0, 4, 9):
        def g_of(h, b=b):
            t = w.t.copy()
            t[b] += h
            return O.brute_gradient(w.parent, t, *args_of(w)[2:])[1][b]
        d = richardson_directional(g_of, h=min(1e-2, w.t[b] / 2), levels=3)
        assert abs(d - nh["hess"][b]) < 1e-7 * nh["abs_hess"][b]


# ---------------------------------------------------------------- input checks


def test_validation_rejects_bad_inputs():
    w = small(n_tips=4)
    a = list(args_of(w))
    bad = []
    p = a[0].copy(); p[0] = p[1] = p[2] = 4; bad.append((0, p))     # non-binary
    p = a[0].copy(); p[-1] = 3; bad.append((0, p))                  # root has a parent
    Q = a[2].copy(); Q[0, 1] = -0.1; bad.append((2, Q))             # negative rate
    Q = a[2].copy(); Q[0, 0] += 0.01; bad.append((2, Q))            # row sum
    bad.append((3, np.array([0.5, 0.5, 0.5, -0.5])))                # pi
    t = a[1].copy(); t[0] = np.nan; bad.append((1, t))
    t = a[1].copy(); t[0] = -1e-3; bad.append((1, t))
    m = a[6].copy(); m[0, 0] = 0; bad.append((6, m))                # empty mask
    m = a[6].copy(); m[0, 0] = np.uint64(1 << 5); bad.append((6, m))  # state beyond m
    ww = a[7].copy(); ww[0] = -1; bad.append((7, ww))
    for pos, val in bad:
        b = list(a)
        b[pos] = val
        with pytest.raises(O.OracleInputError):
            O.log_likelihood(*b)


def test_fig1_three_taxon_worked_example():
    """Fig. 1: P(Y) = pi^T [P_4 (P_1 p_1 o P_2 p_2) o P_3 p_3] and
    q_4 = P_4^T [q_5 o (P_3 p_3)], with q_4^T p_4 = P(Y) (0-based labels)."""
    rng = np.random.default_rng(11)
    Q = random_rate_matrix(4, rng)
    pi = rng.dirichlet(np.ones(4))
    parent = np.array([3, 3, 4, 4, -1])
    t = np.array([0.1, 0.2, 0.3, 0.15])
    y = np.array([[0], [2], [1]], dtype=np.int16)
    masks = states_to_masks(y, 4)
    P = [expm(Q * ti) for ti in t]
    e = np.eye(4)
    p1, p2, p3 = e[0], e[2], e[1]
    p4 = (P[0] @ p1) * (P[1] @ p2)
    lik = pi @ ((P[3] @ p4) * (P[2] @ p3))
    got = O.site_log_likelihoods(parent, t, Q, pi, [1.0], [1.0], masks, [1.0])
    assert abs(got[0] - np.log(lik)) < 1e-14
    q4 = P[3].T @ (pi * (P[2] @ p3))
    assert abs(q4 @ p4 - lik) < 1e-15
    p, lsp, q, lsq = O.linear_partials(parent, t, Q, pi, [1.0], [1.0], masks, [1.0])
    q4_oracle = q[3][0, 0] * np.exp(lsq[3][0])
    assert np.abs(q4_oracle - q4).max() < 1e-15


def test_linear_hessian_magnitude_bounds_the_hessian():
    w = small(n_tips=9, n_cats=3, n_patterns=20, seed=44)
    lin = O.linear_gradient(*args_of(w))
    nh = O.naive_hessian_diag(*args_of(w))
    assert (np.abs(lin["hess"]) <= lin["abs_hess"] * (1 + 1e-12)).all()
    assert np.allclose(lin["abs_hess"], nh["abs_hess"], rtol=1e-11, atol=0)
