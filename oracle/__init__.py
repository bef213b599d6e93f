"""CPU FP64 oracle for the phylogenetic log-likelihood and its branch gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library
never links or calls it, and it shares no code with the GPU path: the only
common inputs come from the seeded generators in ``synth``.

What it computes (Ji et al., "Gradients do grow on trees", Section 2):
  * ``brute``    -- the likelihood of Eq. (likelihood) by enumerating every
                    latent internal state, and its exact derivative;
  * ``pruning``  -- Felsenstein's post-order pruning, Eqs. (pruning),
                    (postOrderPartialUpdate), (rootInnerProduct) and
                    (discreteRateLikelihood), with per-site rescaling;
  * ``naive``    -- the O(N^2) gradient that re-runs pruning once per branch
                    with dP/dt in place of P (Section 1), and the same for
                    the second derivative;
  * ``linear``   -- the paper's O(N) pre-order pass, Eqs. (preOrderUpdate),
                    (forwardBackwardLikelihood), (singleRateCaseGradient),
                    (GradientWithGamma) and (Hessian), kept as a second,
                    independently pinned route;
  * ``fd``       -- central finite differences (Section 5.1's "Numeric").

Every function is pinned by the CPU tests (tests/test_oracle_*.py) against
brute force, closed forms, invariants or finite differences.  No function
here is "parity unpinned".
"""
from .inputs import Model, Tree, validate, OracleInputError  # noqa: F401
from .transition import transition_matrices, transition_derivatives  # noqa: F401
from .brute import brute_site_likelihoods, brute_gradient  # noqa: F401
from .pruning import site_log_likelihoods, log_likelihood  # noqa: F401
from .naive import naive_gradient, naive_hessian_diag  # noqa: F401
from .linear import linear_gradient, linear_partials  # noqa: F401
from .fd import central_fd_gradient, richardson_directional  # noqa: F401
from .compare import parity_report  # noqa: F401
