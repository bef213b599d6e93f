"""The paper's O(N) gradient: post-order then pre-order (Sections 2.3-2.7).

Post-order (Eq. postOrderPartialUpdate):  p_k = (P_i p_i) o (P_j p_j).
Pre-order  (Eq. preOrderUpdate):          q_root = pi,
                                          q_i = P_i^T [q_k o (P_j p_j)],
for every child i of k with sibling j, tips included.
At every node, per site, q_k^T p_k = P(Y) (Eq. forwardBackwardLikelihood),
and with rate categories (Eqs. discreteRateLikelihood, GradientWithGamma)
    dlogL_s/dt_i = sum_l gamma_l Pr(gamma_l) p_{i|l}^T Q^T q_{i|l}
                   / sum_l Pr(gamma_l) p_{i|l}^T q_{i|l},
    d2logL_s/dt_i^2 = sum_l gamma_l^2 Pr(gamma_l) p^T (Q^2)^T q / (same)
                      - (dlogL_s/dt_i)^2                     (Eq. Hessian).
Both vectors are rescaled per node and site (one factor shared by the
categories); the local ratio cancels the factors.  The cumulative log-scale
of each vector is kept so tests can check the per-node likelihood identity.
"""
from __future__ import annotations

import math

import numpy as np

from .inputs import validate
from .transition import transition_matrices


def _rescale(v):
    c = np.abs(v).max(axis=(0, 2))
    c = np.where(c > 0, c, 1.0)
    return v / c[None, :, None], np.log(c)


def _passes(tree, model, tips, P):
    K, m = len(model.rates), model.m
    S = tips.shape[1]
    p, lsp = {}, {}
    for b in range(tree.n_tips):
        p[b] = np.broadcast_to(tips[b][None, :, :], (K, S, m)).copy()
        lsp[b] = np.zeros(S)
    msg = {}
    for k in tree.postorder():
        i, j = tree.children[k]
        msg[i] = np.matmul(p[i], np.transpose(P[i], (0, 2, 1)))
        msg[j] = np.matmul(p[j], np.transpose(P[j], (0, 2, 1)))
        p[k], c = _rescale(msg[i] * msg[j])
        lsp[k] = lsp[i] + lsp[j] + c
    q, lsq = {}, {}
    q[tree.root] = np.broadcast_to(model.pi[None, None, :], (K, S, m)).copy()
    lsq[tree.root] = np.zeros(S)
    for k in tree.preorder():
        i, j = tree.children[k]
        for a, sib in ((i, j), (j, i)):
            u = q[k] * msg[sib]
            # P^T u: (P^T u)_y = sum_x P[x, y] u[x]  ->  u @ P
            q[a], c = _rescale(np.matmul(u, P[a]))
            lsq[a] = lsq[k] + lsp[sib] + c
    return p, lsp, q, lsq


def linear_partials(parent, t, Q, pi, rates, cat_weights, masks, weights):
    """Scaled post/pre-order vectors of every node and their log-scales.

    Returns (p, log_scale_p, q, log_scale_q), dicts keyed by node, vectors
    shaped [K, S, m]; the unscaled vector is v * exp(log_scale)[None, :, None].
    """
    tree, model, tips, t, _ = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    P = transition_matrices(model.Q, model.rates, t)
    return _passes(tree, model, tips, P)


def linear_gradient(parent, t, Q, pi, rates, cat_weights, masks, weights):
    """dict(logL, grad, abs_grad, hess, abs_hess, site_log_likelihoods) by the O(N) passes.

    abs_hess[i] = sum_s w_s (|d2L_s/L_s| + (dL_s/L_s)^2) bounds |hess[i]| and
    scales its tolerance the way abs_grad does for the gradient."""
    tree, model, tips, t, w = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    P = transition_matrices(model.Q, model.rates, t)
    p, lsp, q, lsq = _passes(tree, model, tips, P)
    root = tree.root
    Ltil = np.einsum("l,lsx,lsx->s", model.cat_weights, p[root], q[root])
    logLs = np.log(Ltil) + lsp[root]
    logL = math.fsum(np.where(w > 0, w * logLs, 0.0).tolist())
    B = tree.n_nodes - 1
    grad, absg, hess, absh = np.zeros(B), np.zeros(B), np.zeros(B), np.zeros(B)
    g1 = model.rates * model.cat_weights
    g2 = model.rates ** 2 * model.cat_weights
    for i in range(B):
        # p^T Q_i^T q = q^T Q_i p, per category and site (Q_i: branch i's matrix)
        Qi = model.Q_of(i)
        Qp = np.matmul(p[i], Qi.T)
        Q2p = np.matmul(p[i], (Qi @ Qi).T)
        den = np.einsum("l,lsx,lsx->s", model.cat_weights, q[i], p[i])
        num = np.einsum("l,lsx,lsx->s", g1, q[i], Qp)
        num2 = np.einsum("l,lsx,lsx->s", g2, q[i], Q2p)
        r1 = num / den
        r2 = num2 / den
        grad[i] = math.fsum((w * r1).tolist())
        absg[i] = math.fsum(np.abs(w * r1).tolist())
        hess[i] = math.fsum((w * (r2 - r1 * r1)).tolist())
        absh[i] = math.fsum((w * (np.abs(r2) + r1 * r1)).tolist())
    return dict(logL=logL, grad=grad, abs_grad=absg, hess=hess, abs_hess=absh, site_log_likelihoods=logLs)
