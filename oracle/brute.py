"""Likelihood by enumeration of latent states (Section 2.2, Eq. likelihood).

For each rate category l (Eq. discreteRateLikelihood) and each site,
  L_{s,l} = sum over all internal-node states y of
            pi[y_root] * prod_{non-root b} Pr(Y_b | Y_pa(b)),
where a tip observed as a set A of allowed states contributes
sum_{y in A} P_{b|l}[y_pa, y] (Section 2.1: partly observed data modify the
tip vector), and L_s = sum_l Pr(gamma_l) L_{s,l}.

The derivative with respect to t_b replaces the factor of branch b by the
same entry of dP_{b|l}/dt_b = gamma_l Q P_{b|l}; the product rule over the
enumerated sum then gives dL_s/dt_b exactly.  Exponential in N: tiny trees only.
"""
from __future__ import annotations

import itertools

import numpy as np

from .inputs import validate
from .transition import transition_derivatives, transition_matrices


def _enumerate(tree, model, tips, t, with_grad):
    N, m = tree.n_tips, model.m
    K = len(model.rates)
    S = tips.shape[1]
    P = transition_matrices(model.Q, model.rates, t)
    dP = transition_derivatives(model.Q, model.rates, P) if with_grad else None
    internal = list(range(N, tree.n_nodes))
    branches = list(range(tree.n_nodes - 1))
    L = np.zeros((K, S))
    dL = np.zeros((len(branches), K, S)) if with_grad else None
    for states in itertools.product(range(m), repeat=len(internal)):
        y = dict(zip(internal, states))
        # factor[b] is an array [K, S] for every branch b
        factor = {}
        dfactor = {}
        for b in branches:
            ya = y[int(tree.parent[b])]
            if b < N:
                # set observation at a tip: sum over the allowed child states
                factor[b] = np.einsum("ky,sy->ks", P[b, :, ya, :], tips[b])
                if with_grad:
                    dfactor[b] = np.einsum("ky,sy->ks", dP[b, :, ya, :], tips[b])
            else:
                yb = y[b]
                factor[b] = np.repeat(P[b, :, ya, yb][:, None], S, axis=1)
                if with_grad:
                    dfactor[b] = np.repeat(dP[b, :, ya, yb][:, None], S, axis=1)
        root_p = model.pi[y[tree.root]]
        prod = np.full((K, S), root_p)
        for b in branches:
            prod = prod * factor[b]
        L += prod
        if with_grad:
            for b in branches:
                term = np.full((K, S), root_p)
                for c in branches:
                    term = term * (dfactor[c] if c == b else factor[c])
                dL[b] += term
    return L, dL


def brute_site_likelihoods(parent, t, Q, pi, rates, cat_weights, masks, weights):
    """Per-site likelihoods L_s (not logs), shape [S]."""
    tree, model, tips, t, _ = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    L, _ = _enumerate(tree, model, tips, t, with_grad=False)
    return model.cat_weights @ L


def brute_gradient(parent, t, Q, pi, rates, cat_weights, masks, weights):
    """(logL, grad[2N-2], L_s[S], dL_s/dt_b [2N-2, S]) by enumeration."""
    tree, model, tips, t, weights = validate(parent, t, Q, pi, rates, cat_weights, masks, weights)
    L, dL = _enumerate(tree, model, tips, t, with_grad=True)
    Ls = model.cat_weights @ L
    dLs = np.einsum("k,bks->bs", model.cat_weights, dL)
    logL = float(np.sum(weights * np.log(Ls)))
    grad = (dLs / Ls[None, :]) @ weights
    return logL, grad, Ls, dLs
