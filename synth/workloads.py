"""Seeded synthetic workloads (trees, CTMC models, alignments).

Every draw uses NumPy's PCG64 generator with a fixed seed, so a workload is
a pure function of (config, overrides).  Nothing here evaluates a
likelihood: site patterns are simulated down the tree with the exact
jump-chain construction of a CTMC (exponential holding times, jumps drawn
from the off-diagonal rates), never with a transition matrix.

Conventions shared by every consumer (Section 2.1 of the paper numbers tips
1..N and internal nodes N+1..2N-1 with the root last; here the same order is
0-based):
  * tips are nodes 0..N-1, internal nodes N..2N-2, the root is 2N-2;
  * internal nodes are labelled in a post-order, so every parent has a larger
    label than its children;
  * ``parent[b]`` is the parent of node b and ``parent[root] == -1``;
  * a branch is named by its child node, so ``t[b]`` (b = 0..2N-3) is the
    length of the branch above node b;
  * ``Q[x, y]`` is the rate from parent state x to child state y (rows sum
    to zero) and the root distribution ``pi`` need not be stationary;
  * tip observations are state indices with -1 for a fully missing state,
    or bit masks (bit x set = state x allowed) from ``states_to_masks``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
from scipy import special

# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

CONFIGS = {
    # small correctness case: 8 tips, 1 category, random tips
    "C1": dict(index=1, n_tips=8, n_states=4, n_cats=1, alpha=None, n_patterns=200,
               mean_t=0.05, tips="uniform", ambiguous_frac=0.05, w_max=10),
    # headline workload: 1000 tips, 4 gamma categories, simulated sites
    "C2": dict(index=2, n_tips=1000, n_states=4, n_cats=4, alpha=0.5, n_patterns=2000,
               mean_t=0.01, tips="simulate", ambiguous_frac=0.0, w_max=20),
    # serving requests: sizes drawn per request (see serving_requests)
    "C3": dict(index=3, n_tips=None, n_states=4, n_cats=4, alpha=0.5, n_patterns=None,
               mean_t=0.01, tips="simulate", ambiguous_frac=0.0, w_max=20),
    # codon model, 61 sense codons
    "C4": dict(index=4, n_tips=256, n_states=61, n_cats=4, alpha=0.5, n_patterns=1000,
               mean_t=0.01, tips="simulate", ambiguous_frac=0.0, w_max=20),
    # amino-acid model with a random-effects clock (t_b = r_b * tau_b)
    "C5": dict(index=5, n_tips=500, n_states=20, n_cats=4, alpha=0.5, n_patterns=3000,
               mean_t=0.01, tips="simulate", ambiguous_frac=0.0, w_max=20),
}


def config_seed(index: int) -> int:
    """Seed of configuration ``index`` (1-based)."""
    return 12146 * 10 + int(index)


@dataclasses.dataclass
class Workload:
    name: str
    parent: np.ndarray          # int32 [2N-1]
    t: np.ndarray               # float64 [2N-2], branch above node b
    Q: np.ndarray               # float64 [m, m]
    pi: np.ndarray              # float64 [m]
    rates: np.ndarray           # float64 [K] category rates gamma_l
    cat_weights: np.ndarray     # float64 [K] Pr(gamma_l)
    tip_states: np.ndarray      # int16 [N, S], -1 = fully ambiguous
    weights: np.ndarray         # float64 [S] pattern weights
    tau: Optional[np.ndarray] = None    # C5: fixed times per branch
    log_r: Optional[np.ndarray] = None  # C5: log branch rates
    masks: Optional[np.ndarray] = None  # uint64 [N, S] tip masks (overrides tip_states)

    @property
    def n_tips(self) -> int:
        return (len(self.parent) + 1) // 2

    @property
    def n_states(self) -> int:
        return self.Q.shape[0]

    @property
    def n_patterns(self) -> int:
        return len(self.weights)

    @property
    def n_cats(self) -> int:
        return len(self.rates)

    def tip_masks(self) -> np.ndarray:
        if self.masks is not None:
            return self.masks
        return states_to_masks(self.tip_states, self.n_states)


# ---------------------------------------------------------------------------
# trees
# ---------------------------------------------------------------------------

def yule_tree(n_tips: int, rng: np.random.Generator) -> np.ndarray:
    """Random rooted binary tree by Yule splitting; returns the parent array.

    Start from a root with two tips, then repeatedly pick a tip uniformly at
    random and give it two children, until there are ``n_tips`` tips.  Nodes
    are relabelled so tips are 0..N-1 (in order of a depth-first walk) and
    internal nodes N..2N-2 in post-order (root last).
    """
    if n_tips < 2:
        raise ValueError("a rooted binary tree needs at least 2 tips")
    children = {0: [1, 2]}
    tips = [1, 2]
    next_id = 3
    while len(tips) < n_tips:
        k = int(rng.integers(len(tips)))
        node = tips[k]
        a, b = next_id, next_id + 1
        next_id += 2
        children[node] = [a, b]
        tips[k] = a
        tips.append(b)
    # iterative post-order walk from the raw root 0
    order = []
    stack = [(0, False)]
    while stack:
        node, expanded = stack.pop()
        if node not in children:
            order.append(node)
        elif expanded:
            order.append(node)
        else:
            stack.append((node, True))
            c0, c1 = children[node]
            stack.append((c1, False))
            stack.append((c0, False))
    label = {}
    n_tip_seen = 0
    n_int_seen = 0
    for node in order:
        if node in children:
            label[node] = n_tips + n_int_seen
            n_int_seen += 1
        else:
            label[node] = n_tip_seen
            n_tip_seen += 1
    parent = np.full(2 * n_tips - 1, -1, dtype=np.int32)
    for node, (c0, c1) in children.items():
        parent[label[c0]] = label[node]
        parent[label[c1]] = label[node]
    assert parent[2 * n_tips - 2] == -1
    return parent


# ---------------------------------------------------------------------------
# substitution models
# ---------------------------------------------------------------------------

def _stationary(Q: np.ndarray) -> np.ndarray:
    """Stationary distribution of a generator: solve pi Q = 0, sum(pi) = 1."""
    m = Q.shape[0]
    A = np.vstack([Q.T, np.ones((1, m))])
    b = np.zeros(m + 1)
    b[-1] = 1.0
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    return sol


def _normalise(Q: np.ndarray) -> np.ndarray:
    """Scale Q to one expected substitution per unit time at stationarity."""
    Q = Q.copy()
    np.fill_diagonal(Q, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    pi_q = _stationary(Q)
    rate = -float(np.dot(pi_q, np.diag(Q)))
    return Q / rate


def random_rate_matrix(m: int, rng: np.random.Generator) -> np.ndarray:
    """Non-reversible generator: off-diagonals ~ Exp(1), rows sum to zero."""
    Q = rng.exponential(1.0, size=(m, m))
    return _normalise(Q)


_BASES = "TCAG"
# standard genetic code, codons enumerated with bases in TCAG order
_AMINO = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"


def sense_codons():
    """The 61 sense codons of the standard genetic code and their amino acids."""
    out = []
    idx = 0
    for a in _BASES:
        for b in _BASES:
            for c in _BASES:
                aa = _AMINO[idx]
                idx += 1
                if aa != "*":
                    out.append((a + b + c, aa))
    return out


def codon_rate_matrix(pi: np.ndarray, kappa: float, omega: float,
                      rng: np.random.Generator, perturb: float = 0.1) -> np.ndarray:
    """61-state codon generator with a random non-reversible perturbation.

    q_xy is non-zero only when codons x and y differ at one position; then it
    is kappa^[transition] * omega^[non-synonymous] * pi_y, multiplied by
    (1 + perturb * U(-1, 1)).
    """
    codons = sense_codons()
    purines = set("AG")
    m = len(codons)
    Q = np.zeros((m, m))
    for x, (cx, ax) in enumerate(codons):
        for y, (cy, ay) in enumerate(codons):
            diff = [i for i in range(3) if cx[i] != cy[i]]
            if len(diff) != 1:
                continue
            i = diff[0]
            transition = (cx[i] in purines) == (cy[i] in purines)
            rate = pi[y]
            if transition:
                rate *= kappa
            if ax != ay:
                rate *= omega
            Q[x, y] = rate
    noise = 1.0 + perturb * rng.uniform(-1.0, 1.0, size=(m, m))
    Q = Q * noise
    return _normalise(Q)


def discrete_gamma(alpha: float, n_cats: int):
    """Mean-of-category discrete gamma rates (Yang 1994) with equal weights.

    Rates are scaled so sum_l w_l * r_l == 1 exactly in floating point terms
    of the returned arrays (up to one rounding).
    """
    if n_cats == 1:
        return np.array([1.0]), np.array([1.0])
    cuts = special.gammaincinv(alpha, np.arange(1, n_cats) / n_cats) / alpha
    upper = np.concatenate([special.gammainc(alpha + 1.0, cuts * alpha), [1.0]])
    lower = np.concatenate([[0.0], special.gammainc(alpha + 1.0, cuts * alpha)])
    rates = n_cats * (upper - lower)
    weights = np.full(n_cats, 1.0 / n_cats)
    rates = rates / float(np.dot(rates, weights))
    return rates, weights


# ---------------------------------------------------------------------------
# alignments
# ---------------------------------------------------------------------------

def simulate_sites(parent: np.ndarray, t: np.ndarray, Q: np.ndarray, pi: np.ndarray,
                   rates: np.ndarray, cat_weights: np.ndarray, n_sites: int,
                   rng: np.random.Generator) -> np.ndarray:
    """Simulate tip states by running the CTMC down every branch.

    Each site draws a root state from ``pi`` and a rate category from
    ``cat_weights``; along a branch of length t and category rate g the chain
    holds in state x for Exp(-Q[x, x] * g) time and then jumps to y with
    probability Q[x, y] / -Q[x, x].  Returns int16 [N, n_sites].
    """
    m = Q.shape[0]
    n_nodes = len(parent)
    n_tips = (n_nodes + 1) // 2
    root = n_nodes - 1
    hold = -np.diag(Q)
    jump = Q.copy()
    np.fill_diagonal(jump, 0.0)
    cdf = np.cumsum(jump, axis=1)
    state = np.empty((n_nodes, n_sites), dtype=np.int16)
    state[root] = rng.choice(m, size=n_sites, p=pi / pi.sum())
    cat = rng.choice(len(rates), size=n_sites, p=cat_weights / cat_weights.sum())
    site_rate = rates[cat]
    # parents carry larger labels than their children: descending order is a pre-order
    for node in range(n_nodes - 2, -1, -1):
        x = state[parent[node]].astype(np.int64)
        remaining = site_rate * t[node]
        active = np.ones(n_sites, dtype=bool)
        while active.any():
            idx = np.nonzero(active)[0]
            h = hold[x[idx]]
            dt = rng.exponential(1.0, size=idx.size) / np.where(h > 0, h, 1.0)
            dt = np.where(h > 0, dt, np.inf)
            jumps = dt < remaining[idx]
            stop = idx[~jumps]
            active[stop] = False
            go = idx[jumps]
            if go.size == 0:
                continue
            remaining[go] -= dt[jumps]
            rows = cdf[x[go]]
            u = (1.0 - rng.random(go.size)) * rows[:, -1]
            x[go] = np.argmax(rows >= u[:, None], axis=1)
        state[node] = x
    return state[:n_tips].copy()


def states_to_masks(tip_states: np.ndarray, n_states: int) -> np.ndarray:
    """State indices (-1 = missing) to uint64 bit masks of allowed states."""
    if n_states > 64:
        raise ValueError("masks hold at most 64 states")
    full = np.uint64((1 << n_states) - 1) if n_states < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    s = tip_states.astype(np.int64)
    masks = np.where(s < 0, full, np.left_shift(np.uint64(1), np.maximum(s, 0).astype(np.uint64)))
    return masks.astype(np.uint64)


# ---------------------------------------------------------------------------
# workload factory
# ---------------------------------------------------------------------------

def make_workload(name: str, seed: Optional[int] = None, **overrides) -> Workload:
    """Build configuration ``name`` ("C1", "C2", "C4", "C5", or "C3" with
    explicit ``n_tips`` and ``n_patterns``), optionally with overrides of
    ``n_tips``, ``n_patterns``, ``n_cats``, ``n_states``, ``alpha``,
    ``mean_t``, ``ambiguous_frac`` and ``tips`` ("uniform" or "simulate")."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    rng = np.random.Generator(np.random.PCG64(config_seed(cfg["index"]) if seed is None else seed))
    n, m, K, S = cfg["n_tips"], cfg["n_states"], cfg["n_cats"], cfg["n_patterns"]
    parent = yule_tree(n, rng)
    tau = log_r = None
    if name == "C5" and cfg.get("clock", True):
        tau = rng.exponential(cfg["mean_t"], size=2 * n - 2)
        log_r = rng.normal(0.0, 0.5, size=2 * n - 2)
        t = np.exp(log_r) * tau
    else:
        t = rng.exponential(cfg["mean_t"], size=2 * n - 2)
    pi = rng.dirichlet(np.ones(m))
    if m == 61:
        kappa = float(rng.lognormal(1.0, 0.3))
        omega = float(rng.lognormal(-1.0, 0.5))
        Q = codon_rate_matrix(pi, kappa, omega, rng)
    else:
        Q = random_rate_matrix(m, rng)
    if cfg["alpha"] is None or K == 1:
        rates, cat_w = discrete_gamma(1.0, 1) if K == 1 else discrete_gamma(1.0, K)
    else:
        rates, cat_w = discrete_gamma(cfg["alpha"], K)
    if cfg["tips"] == "uniform":
        tip_states = rng.integers(0, m, size=(n, S)).astype(np.int16)
    else:
        tip_states = simulate_sites(parent, t, Q, pi, rates, cat_w, S, rng)
    if cfg["ambiguous_frac"] > 0:
        miss = rng.random((n, S)) < cfg["ambiguous_frac"]
        tip_states = np.where(miss, -1, tip_states).astype(np.int16)
    weights = rng.integers(1, cfg["w_max"] + 1, size=S).astype(np.float64)
    return Workload(name=name, parent=parent, t=t, Q=Q, pi=pi, rates=rates,
                    cat_weights=cat_w, tip_states=tip_states, weights=weights,
                    tau=tau, log_r=log_r)


@dataclasses.dataclass
class RequestSpec:
    rid: int
    arrival_s: float
    n_tips: int
    n_patterns: int
    seed: int


def serving_requests(n_requests: int = 256, qps: float = 10.0, seed: Optional[int] = None,
                     n_tips_range=(100, 2000), n_patterns_range=(500, 5000)) -> List[RequestSpec]:
    """Poisson arrivals of requests with N ~ U{100..2000}, S ~ U{500..5000}."""
    rng = np.random.Generator(np.random.PCG64(config_seed(3) if seed is None else seed))
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        out.append(RequestSpec(
            rid=r, arrival_s=float(arrivals[r]),
            n_tips=int(rng.integers(n_tips_range[0], n_tips_range[1] + 1)),
            n_patterns=int(rng.integers(n_patterns_range[0], n_patterns_range[1] + 1)),
            seed=int(rng.integers(1 << 62))))
    return out


def request_workload(spec: RequestSpec) -> Workload:
    """The workload of one serving request."""
    return make_workload("C3", seed=spec.seed, n_tips=spec.n_tips, n_patterns=spec.n_patterns)


def perturb_lengths(t: np.ndarray, rng: np.random.Generator, scale: float = 0.01) -> np.ndarray:
    """Next branch lengths of a request: t * exp(scale * N(0, 1))."""
    return t * np.exp(scale * rng.normal(size=t.shape))


def branch_models(workload: Workload, n_models: int, seed: int = 0):
    """A non-homogeneous model for a workload: n_models random non-reversible
    rate matrices (the first is the workload's Q) and a model index per
    branch, uniform over the models.  Returns (Qs [n_models, m, m],
    model_of_branch int32 [2N-2])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = workload.n_states
    Qs = [workload.Q] + [random_rate_matrix(m, rng) for _ in range(n_models - 1)]
    model = rng.integers(0, n_models, size=len(workload.t)).astype(np.int32)
    return np.stack(Qs), model
