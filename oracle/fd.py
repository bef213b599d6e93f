"""Central finite differences of the log-likelihood (Section 5.1, "Numeric").

g_b ~ [logL(t + h e_b) - logL(t - h e_b)] / (2h), two pruning passes per
branch.  ``richardson_directional`` extrapolates a central difference along a
direction to higher order, for identities such as d/dc logL(c t) at c = 1.
"""
from __future__ import annotations

import numpy as np

from .pruning import log_likelihood


def central_fd_gradient(parent, t, Q, pi, rates, cat_weights, masks, weights, h=1e-6,
                        branches=None):
    t = np.asarray(t, dtype=np.float64)
    B = len(t)
    if branches is None:
        branches = range(B)
    g = np.full(B, np.nan)
    for b in branches:
        tp = t.copy()
        tm = t.copy()
        tp[b] += h
        tm[b] -= h
        if tm[b] < 0:
            raise ValueError("central difference needs t_b >= h")
        fp = log_likelihood(parent, tp, Q, pi, rates, cat_weights, masks, weights)
        fm = log_likelihood(parent, tm, Q, pi, rates, cat_weights, masks, weights)
        g[b] = (fp - fm) / (2 * h)
    return g


def richardson_directional(f, h=1e-2, levels=4):
    """d/dx f at x = 0 by Richardson-extrapolated central differences."""
    table = []
    for n in range(levels):
        hn = h / (2 ** n)
        row = [(f(hn) - f(-hn)) / (2 * hn)]
        for j in range(1, n + 1):
            prev = table[n - 1][j - 1]
            row.append(row[j - 1] + (row[j - 1] - prev) / (4 ** j - 1))
        table.append(row)
    return table[-1][-1]
