"""Pins of the parity rule every GPU test goes through (oracle.compare) and of
the cancellation-free gradient magnitude A_b it divides by.

The rule (per-site derivative of Section 2.5, summed over sites with the
rate categories of Section 2.6, Eq. GradientWithGamma): a result passes when
|logL - logL*| <= tol |logL*| and, for every branch, |g_b - g*_b| <= tol A_b
with A_b = sum_s w_s |d log L_s / dt_b|.  These tests fix the rule from
outside: a result off by twice the tolerance on a single branch, a NaN or
a logL off by twice the tolerance must fail; one off by half of it must pass;
and A_b must equal the sum over sites of |g_b| of one-site alignments,
which the oracle computes by separate calls.
"""
import numpy as np
import pytest

import oracle as O
from synth import states_to_masks
from tests._fixtures import args_of, small


def _reference(n_tips=6, n_patterns=30, n_cats=2, seed=11):
    w = small(n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats, seed=seed)
    ref = O.naive_gradient(*args_of(w))
    return w, ref


@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_exact_result_passes_and_reports_every_branch(tol):
    _, ref = _reference()
    rep = O.parity_report(ref["logL"], ref["grad"].copy(), ref["logL"], ref["grad"], ref["abs_grad"], tol)
    assert rep["ok"]
    assert rep["n_checked"] == len(ref["grad"])
    assert rep["grad_rel_A_max"] == 0.0 and rep["logL_rel"] == 0.0


@pytest.mark.parametrize("tol", [1e-10, 1e-5])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_one_branch_off_by_twice_the_tolerance_fails(tol, sign):
    _, ref = _reference()
    B = len(ref["grad"])
    for b in (0, B // 2, B - 1):
        g = ref["grad"].copy()
        g[b] += sign * 2.0 * tol * ref["abs_grad"][b]
        rep = O.parity_report(ref["logL"], g, ref["logL"], ref["grad"], ref["abs_grad"], tol)
        assert not rep["ok"], (b, rep)
        assert rep["grad_rel_A_max"] == pytest.approx(2.0 * tol, rel=1e-3)


@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_every_branch_off_by_half_the_tolerance_passes(tol):
    _, ref = _reference()
    rng = np.random.default_rng(3)
    signs = rng.choice([-1.0, 1.0], size=len(ref["grad"]))
    g = ref["grad"] + signs * 0.5 * tol * ref["abs_grad"]
    logL = ref["logL"] * (1.0 + 0.5 * tol)
    rep = O.parity_report(logL, g, ref["logL"], ref["grad"], ref["abs_grad"], tol)
    assert rep["ok"], rep


@pytest.mark.parametrize("tol", [1e-10, 1e-5])
def test_logL_off_by_twice_the_tolerance_fails(tol):
    _, ref = _reference()
    for f in (1.0 + 2.0 * tol, 1.0 - 2.0 * tol):
        rep = O.parity_report(ref["logL"] * f, ref["grad"].copy(), ref["logL"], ref["grad"], ref["abs_grad"], tol)
        assert not rep["ok"], rep


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_values_fail(bad):
    _, ref = _reference()
    g = ref["grad"].copy()
    g[2] = bad
    assert not O.parity_report(ref["logL"], g, ref["logL"], ref["grad"], ref["abs_grad"], 1e-5)["ok"]
    assert not O.parity_report(bad, ref["grad"].copy(), ref["logL"], ref["grad"], ref["abs_grad"], 1e-5)["ok"]


def test_cancelling_branch_is_measured_against_A_not_against_g():
    # a branch whose site terms cancel (|g| << A): half the tolerance of A
    # passes although it is far beyond tol relative to g; twice fails
    ref_g = np.array([1e-4, 2.0])
    ref_a = np.array([1.0, 2.0])
    tol = 1e-10
    ok = O.parity_report(-100.0, ref_g + np.array([0.5 * tol, 0.0]), -100.0, ref_g, ref_a, tol)
    bad = O.parity_report(-100.0, ref_g + np.array([2.0 * tol, 0.0]), -100.0, ref_g, ref_a, tol)
    assert ok["ok"] and ok["grad_rel_plain_max"] > 100 * tol
    assert not bad["ok"]
    assert ok["n_cancelling"] == 1


def test_subset_of_branches_checks_only_those():
    _, ref = _reference()
    g = ref["grad"].copy()
    g[0] = np.nan
    rep = O.parity_report(ref["logL"], g, ref["logL"], ref["grad"], ref["abs_grad"], 1e-10, branches=[1, 2, 3])
    assert rep["ok"] and rep["n_checked"] == 3


# ---------------------------------------------------------------- the magnitude A_b


@pytest.mark.parametrize("route", ["naive", "linear"])
def test_A_bounds_the_gradient_on_every_branch(route):
    w, _ = _reference(n_tips=7, n_patterns=60, n_cats=3, seed=5)
    res = O.naive_gradient(*args_of(w)) if route == "naive" else O.linear_gradient(*args_of(w))
    assert np.all(res["abs_grad"] >= np.abs(res["grad"]))
    # with 60 sites of both signs some branch cancels
    assert np.any(res["abs_grad"] > 1.5 * np.abs(res["grad"]))


@pytest.mark.parametrize("route", ["naive", "linear"])
def test_A_equals_abs_gradient_for_a_single_site(route):
    w, _ = _reference(n_tips=6, n_patterns=1, n_cats=2, seed=9)
    res = O.naive_gradient(*args_of(w)) if route == "naive" else O.linear_gradient(*args_of(w))
    assert np.array_equal(res["abs_grad"], np.abs(res["grad"]))


@pytest.mark.parametrize("route", ["naive", "linear"])
def test_A_is_the_sum_of_one_site_gradient_magnitudes(route):
    # A_b of an alignment = sum over its sites s of |g_b| of the alignment
    # made of site s alone (with weight w_s): each one-site gradient is a
    # separate oracle call, so an inflated, deflated or unweighted A fails
    w, _ = _reference(n_tips=6, n_patterns=12, n_cats=2, seed=4)
    fn = O.naive_gradient if route == "naive" else O.linear_gradient
    full = fn(*args_of(w))
    masks = w.tip_masks()
    tot = np.zeros_like(full["grad"])
    for s in range(len(w.weights)):
        one = fn(w.parent, w.t, w.Q, w.pi, w.rates, w.cat_weights, masks[:, s:s + 1], w.weights[s:s + 1])
        tot += np.abs(one["grad"])
    assert np.allclose(full["abs_grad"], tot, rtol=1e-12, atol=0.0)


def test_A_scales_with_the_site_weights():
    # doubling every weight doubles g and A; the rule's outcome is unchanged
    w, _ = _reference(n_tips=5, n_patterns=8, n_cats=1, seed=2)
    a = O.naive_gradient(*args_of(w))
    w2 = args_of(w)[:-1] + (2.0 * w.weights,)
    b = O.naive_gradient(*w2)
    assert np.allclose(b["abs_grad"], 2.0 * a["abs_grad"], rtol=1e-14)
    assert np.allclose(b["grad"], 2.0 * a["grad"], rtol=1e-13, atol=1e-13 * a["abs_grad"].max())


def test_one_hot_masks_helper_roundtrip():
    # the masks the one-site calls above slice are the alignment's own
    states = np.array([[0, 3, -1], [2, 1, 0]], dtype=np.int16)
    m = states_to_masks(states, 4)
    assert m[0, 0] == 1 and m[0, 1] == 8 and m[0, 2] == 15 and m[1, 0] == 4
