"""Small helpers shared by the tests: workload argument tuples and tiny models."""
import numpy as np

from synth import make_workload, states_to_masks


def args_of(w):
    return (w.parent, w.t, w.Q, w.pi, w.rates, w.cat_weights, w.tip_masks(), w.weights)


def small(n_tips=5, n_patterns=40, n_cats=1, n_states=4, seed=7, ambiguous=0.1, alpha=0.5,
          tips="uniform", mean_t=0.1):
    return make_workload("C1", seed=seed, n_tips=n_tips, n_patterns=n_patterns, n_cats=n_cats,
                         n_states=n_states, ambiguous_frac=ambiguous, alpha=alpha, tips=tips,
                         mean_t=mean_t)


def jc_matrix(m=4):
    """Unit-rate Jukes-Cantor generator: q_xy = 1/(m-1), q_xx = -1."""
    Q = np.full((m, m), 1.0 / (m - 1))
    np.fill_diagonal(Q, -1.0)
    return Q


def gtr_matrix(rng, m=4):
    """A reversible generator with stationary distribution pi (Q = S diag(pi))."""
    pi = rng.dirichlet(np.ones(m))
    S = rng.exponential(1.0, size=(m, m))
    S = (S + S.T) / 2
    Q = S * pi[None, :]
    np.fill_diagonal(Q, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    return Q, pi


def all_patterns(n_tips, m):
    """Every one of the m^N fully observed tip patterns, as masks [N, m^N]."""
    grid = np.stack(np.meshgrid(*[np.arange(m)] * n_tips, indexing="ij"), 0).reshape(n_tips, -1)
    return states_to_masks(grid.astype(np.int16), m)
