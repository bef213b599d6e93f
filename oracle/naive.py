"""The O(N^2) gradient by repeated pruning (Section 1).

dL_s/dt_b is the pruning recursion with P_{b|l} replaced by its derivative
gamma_l Q P_{b|l}; one full post-order pass per branch.  The log-likelihood
gradient is then
    g_b = sum_s w_s (dL_s/dt_b) / L_s,
and A_b = sum_s w_s |(dL_s/dt_b) / L_s| is its cancellation-free magnitude,
used to state a relative tolerance that stays meaningful when g_b ~ 0.
The second derivative (Section 2.7, per site) substitutes
gamma_l^2 Q^2 P_{b|l}:
    H_b = sum_s w_s [ (d2L_s/dt_b^2) / L_s - ((dL_s/dt_b) / L_s)^2 ].
Site sums use math.fsum (exactly rounded).
"""
from __future__ import annotations

import math

import numpy as np

from .inputs import validate
from .pruning import prune
from .transition import transition_derivatives, transition_matrices


def _site_ratios(tree, model, tips, P, D, b, root0, ls0):
    mats = P.copy()
    mats[b] = D[b]
    root_b, ls_b = prune(tree, model, tips, mats, rescale=True)
    num = model.cat_weights @ root_b
    den = model.cat_weights @ root0
    return (num / den) * np.exp(ls_b - ls0)


def naive_gradient(parent, t, Q, pi, rates, cat_weights, masks, weights, branches=None):
    """Return dict(logL, grad, abs_grad, branches, site_terms).

    ``branches`` limits the work to a subset (others are NaN); ``site_terms``
    holds w_s * ratio_s for each computed branch, shape [len(branches), S].
    """
    tree, model, tips, t, w = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    P = transition_matrices(model.Q, model.rates, t)
    D = transition_derivatives(model.Q, model.rates, P, order=1)
    root0, ls0 = prune(tree, model, tips, P, rescale=True)
    logLs = np.log(model.cat_weights @ root0) + ls0
    logL = math.fsum(np.where(w > 0, w * logLs, 0.0).tolist())
    B = tree.n_nodes - 1
    if branches is None:
        branches = list(range(B))
    grad = np.full(B, np.nan)
    absg = np.full(B, np.nan)
    terms = np.zeros((len(branches), len(w)))
    for n, b in enumerate(branches):
        r = _site_ratios(tree, model, tips, P, D, b, root0, ls0)
        terms[n] = w * r
        grad[b] = math.fsum(terms[n].tolist())
        absg[b] = math.fsum(np.abs(terms[n]).tolist())
    return dict(logL=logL, grad=grad, abs_grad=absg, branches=list(branches),
                site_terms=terms, site_log_likelihoods=logLs)


def naive_hessian_diag(parent, t, Q, pi, rates, cat_weights, masks, weights, branches=None):
    """Diagonal of the Hessian of logL in the branch lengths, dict(hess, abs_hess, branches)."""
    tree, model, tips, t, w = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    P = transition_matrices(model.Q, model.rates, t)
    D1 = transition_derivatives(model.Q, model.rates, P, order=1)
    D2 = transition_derivatives(model.Q, model.rates, P, order=2)
    root0, ls0 = prune(tree, model, tips, P, rescale=True)
    B = tree.n_nodes - 1
    if branches is None:
        branches = list(range(B))
    hess = np.full(B, np.nan)
    absh = np.full(B, np.nan)
    for b in branches:
        r1 = _site_ratios(tree, model, tips, P, D1, b, root0, ls0)
        r2 = _site_ratios(tree, model, tips, P, D2, b, root0, ls0)
        terms = w * (r2 - r1 * r1)
        hess[b] = math.fsum(terms.tolist())
        absh[b] = math.fsum((w * (np.abs(r2) + r1 * r1)).tolist())
    return dict(hess=hess, abs_hess=absh, branches=list(branches))
