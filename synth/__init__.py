"""Seeded synthetic workloads for the linear-time phylogenetic gradient.

This package only *draws* inputs: trees, branch lengths, rate matrices,
root frequencies, rate categories, weights and tip observations.  It holds
none of the likelihood or gradient arithmetic.  Sites are simulated down
the tree by exact jump-chain (Gillespie) simulation of the CTMC, so the
generator never forms a transition matrix exp(Qt).

Both the CPU oracle (tests only) and the GPU path (tests, bench, smoke)
consume these inputs; nothing else is shared between them.
"""
from .workloads import (  # noqa: F401
    Workload,
    CONFIGS,
    make_workload,
    yule_tree,
    random_rate_matrix,
    codon_rate_matrix,
    discrete_gamma,
    simulate_sites,
    states_to_masks,
    serving_requests,
    request_workload,
    perturb_lengths,
    RequestSpec,
    sense_codons,
    config_seed,
)
