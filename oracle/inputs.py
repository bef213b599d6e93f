"""Oracle input checks and plain containers.

The tree follows Section 2.1: a rooted binary tree, tips first, the root
last, a branch named by its child node.  The model follows Sections 2.1 and
2.6: one rate matrix Q, a root distribution pi that need not be stationary,
and discrete rate categories with rates gamma_l and weights Pr(gamma_l).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


class OracleInputError(ValueError):
    pass


@dataclasses.dataclass
class Tree:
    parent: np.ndarray            # [2N-1], parent[root] == -1
    children: List[List[int]]     # children[k] for every node (empty for tips)
    n_tips: int

    @property
    def n_nodes(self) -> int:
        return len(self.parent)

    @property
    def root(self) -> int:
        return self.n_nodes - 1

    def postorder(self) -> List[int]:
        """Internal nodes, every node after its descendants (Section 2.3)."""
        out = []

        def visit(k):
            for c in self.children[k]:
                visit(c)
            if self.children[k]:
                out.append(k)
        visit(self.root)
        return out

    def preorder(self) -> List[int]:
        """Internal nodes, every node before its descendants (Section 2.4)."""
        return list(reversed(self.postorder()))


@dataclasses.dataclass
class Model:
    Q: np.ndarray            # [m, m], Q[x, y] = rate parent x -> child y; or
                             # [2N-2, m, m], the rate matrix of each branch
    pi: np.ndarray           # [m]
    rates: np.ndarray        # [K] gamma_l
    cat_weights: np.ndarray  # [K] Pr(gamma_l)

    @property
    def m(self) -> int:
        return self.Q.shape[-1]

    def Q_of(self, b: int) -> np.ndarray:
        """Rate matrix on branch b (the branch above node b)."""
        return self.Q[b] if self.Q.ndim == 3 else self.Q


def make_tree(parent) -> Tree:
    parent = np.asarray(parent, dtype=np.int64)
    n_nodes = len(parent)
    if n_nodes < 3 or n_nodes % 2 == 0:
        raise OracleInputError("a rooted binary tree has 2N-1 >= 3 nodes")
    n_tips = (n_nodes + 1) // 2
    root = n_nodes - 1
    if parent[root] != -1:
        raise OracleInputError("the last node must be the root")
    children = [[] for _ in range(n_nodes)]
    for v in range(n_nodes - 1):
        p = int(parent[v])
        if p < n_tips or p >= n_nodes or p == v:
            raise OracleInputError(f"node {v} has an invalid parent {p}")
        children[p].append(v)
    for k in range(n_nodes):
        if k < n_tips and children[k]:
            raise OracleInputError(f"tip {k} has children")
        if k >= n_tips and len(children[k]) != 2:
            raise OracleInputError(f"internal node {k} is not binary")
    # every node must reach the root (no cycles)
    for v in range(n_nodes):
        seen = 0
        u = v
        while u != root:
            u = int(parent[u])
            seen += 1
            if seen > n_nodes:
                raise OracleInputError("the parent array has a cycle")
    return Tree(parent=parent, children=children, n_tips=n_tips)


def validate(parent, t, Q, pi, rates, cat_weights, masks, weights):
    """Check every input; return (Tree, Model, indicator tips [N, S, m])."""
    tree = make_tree(parent)
    Q = np.asarray(Q, dtype=np.float64)
    m = Q.shape[-1]
    if Q.ndim == 3:
        # a non-homogeneous model: one rate matrix per branch (Section 2.1
        # allows the CTMC to differ between branches)
        if Q.shape != (tree.n_nodes - 1, m, m) or m < 2:
            raise OracleInputError("per-branch Q must be [2N-2, m, m]")
    elif Q.shape != (m, m) or m < 2:
        raise OracleInputError("Q must be square with m >= 2")
    for Qb in (Q if Q.ndim == 3 else [Q]):
        off = Qb - np.diag(np.diag(Qb))
        if (off < 0).any():
            raise OracleInputError("off-diagonal rates must be non-negative")
        scale = max(np.abs(Qb).max(), 1.0)
        if np.abs(Qb.sum(axis=1)).max() > 1e-12 * scale * m:
            raise OracleInputError("rows of Q must sum to zero")
    pi = np.asarray(pi, dtype=np.float64)
    if pi.shape != (m,) or (pi < 0).any() or abs(pi.sum() - 1.0) > 1e-12:
        raise OracleInputError("pi must be a probability vector")
    rates = np.asarray(rates, dtype=np.float64)
    cat_weights = np.asarray(cat_weights, dtype=np.float64)
    if rates.ndim != 1 or rates.shape != cat_weights.shape or len(rates) < 1:
        raise OracleInputError("rates and weights must be vectors of equal length")
    if (rates < 0).any() or (cat_weights < 0).any() or abs(cat_weights.sum() - 1.0) > 1e-12:
        raise OracleInputError("category rates >= 0 and weights a probability vector")
    t = np.asarray(t, dtype=np.float64)
    if t.shape != (tree.n_nodes - 1,) or not np.isfinite(t).all() or (t < 0).any():
        raise OracleInputError("branch lengths must be finite and >= 0")
    masks = np.asarray(masks, dtype=np.uint64)
    if masks.ndim != 2 or masks.shape[0] != tree.n_tips:
        raise OracleInputError("tip masks must be [N, S]")
    weights = np.asarray(weights, dtype=np.float64)
    if weights.shape != (masks.shape[1],) or (weights < 0).any() or not np.isfinite(weights).all():
        raise OracleInputError("pattern weights must be finite and >= 0")
    bits = ((masks[:, :, None] >> np.arange(m, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    if m < 64 and (masks >> np.uint64(m)).any():
        raise OracleInputError("tip mask names a state beyond m")
    if (bits.sum(axis=2) == 0).any():
        raise OracleInputError("empty tip mask")
    return tree, Model(Q=Q, pi=pi, rates=rates, cat_weights=cat_weights), bits, t, weights
