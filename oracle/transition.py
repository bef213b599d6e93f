"""Transition matrices of the CTMC (Sections 2.1 and 2.6).

P_{b|l} = exp(Q * gamma_l * t_b), rows indexed by the parent state and
columns by the child state, so P[x, y] = Pr(child = y | parent = x) and each
row sums to one.  The derivative with respect to the branch length is
gamma_l * Q * P_{b|l} (Eq. preOrderPartialGradient uses e^{Qt} Q = Q e^{Qt}).

The matrix exponential is SciPy's scaling-and-squaring Pade routine; the
GPU path uses its own, different method.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def _per_branch(Q, B):
    """Q as [B, m, m]: one matrix repeated, or already one per branch."""
    Q = np.asarray(Q, dtype=np.float64)
    return Q if Q.ndim == 3 else np.broadcast_to(Q, (B,) + Q.shape)


def transition_matrices(Q, rates, t):
    """P[b, l] = expm(Q_b * rates[l] * t[b]); shape [B, K, m, m].  Q is one
    [m, m] matrix or one per branch, [B, m, m]."""
    B, K = len(t), len(rates)
    Qb = _per_branch(Q, B)
    m = Qb.shape[-1]
    P = np.empty((B, K, m, m))
    for b in range(B):
        for l in range(K):
            P[b, l] = expm(Qb[b] * (rates[l] * t[b]))
    return P


def transition_derivatives(Q, rates, P, order=1):
    """d^order/dt^order P[b, l] = (gamma_l Q_b)^order P[b, l]; shape [B, K, m, m]."""
    Qb = _per_branch(Q, P.shape[0])
    Qk = np.stack([np.linalg.matrix_power(q, order) for q in Qb])
    out = np.empty_like(P)
    for l in range(len(rates)):
        out[:, l] = (rates[l] ** order) * np.einsum("bxy,byz->bxz", Qk, P[:, l])
    return out
