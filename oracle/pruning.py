"""Felsenstein pruning: the post-order pass (Section 2.3).

For an internal node k with children i and j (Eq. postOrderPartialUpdate)
    p_k = (P_i p_i) o (P_j p_j),
per rate category (Section 2.6), tip vectors being the indicator of the
allowed states (Section 2.1).  The site likelihood is
    L_s = sum_l Pr(gamma_l) pi^T p_{root|l}        (Eqs. rootInnerProduct and
                                                   discreteRateLikelihood).
Rescaling (not in the paper): after each internal node the site's vectors
are divided by their largest magnitude over categories and states, and the
log of that divisor is added to the site's log-scale, so
    log L_s = log(sum_l Pr(gamma_l) pi^T p~_{root|l}) + log-scale_s.
``prune`` takes the matrices to apply on each branch as an argument so the
naive gradient can substitute dP/dt for one branch (signed values are
rescaled by magnitude the same way).
"""
from __future__ import annotations

import math

import numpy as np

from .inputs import validate
from .transition import transition_matrices


def prune(tree, model, tips, mats, rescale=True):
    """Post-order pass with per-branch matrices ``mats`` [B, K, m, m].

    Returns (root [K, S]: pi^T p~_root per category, log_scale [S]).
    """
    K = len(model.rates)
    S = tips.shape[1]
    p = {}
    for b in range(tree.n_tips):
        p[b] = np.broadcast_to(tips[b][None, :, :], (K, S, model.m))
    log_scale = np.zeros(S)
    for k in tree.postorder():
        i, j = tree.children[k]
        # (P p)_x = sum_y P[x, y] p[y]  ->  p @ P^T, batched over categories
        msg_i = np.matmul(p[i], np.transpose(mats[i], (0, 2, 1)))
        msg_j = np.matmul(p[j], np.transpose(mats[j], (0, 2, 1)))
        pk = msg_i * msg_j
        if rescale:
            c = np.abs(pk).max(axis=(0, 2))
            c = np.where(c > 0, c, 1.0)
            pk = pk / c[None, :, None]
            log_scale = log_scale + np.log(c)
        p[k] = pk
    root = np.einsum("x,ksx->ks", model.pi, p[tree.root])
    return root, log_scale


def site_log_likelihoods(parent, t, Q, pi, rates, cat_weights, masks, weights, rescale=True):
    """log L_s for every site pattern, shape [S]."""
    tree, model, tips, t, _ = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    P = transition_matrices(model.Q, model.rates, t)
    root, log_scale = prune(tree, model, tips, P, rescale=rescale)
    with np.errstate(divide="ignore"):
        return np.log(model.cat_weights @ root) + log_scale


def log_likelihood(parent, t, Q, pi, rates, cat_weights, masks, weights, rescale=True):
    """logL = sum_s w_s log L_s, summed exactly rounded (math.fsum)."""
    ll = site_log_likelihoods(parent, t, Q, pi, rates, cat_weights, masks, weights, rescale)
    w = np.asarray(weights, dtype=np.float64)
    terms = np.where(w > 0, w * ll, 0.0)
    return math.fsum(terms.tolist())
