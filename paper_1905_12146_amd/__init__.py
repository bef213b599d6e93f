"""MI355X-native linear-time phylogenetic log-likelihood gradient.

The GPU work lives in ``libphylograd.so`` (HIP, gfx950) behind the C-ABI of
include/phylograd.h; ``binding`` marshals NumPy arrays and device addresses
into it.  Nothing in this package computes a likelihood on the CPU.
"""
from .binding import (  # noqa: F401
    Context,
    PhyloGradError,
    PG_FP32,
    PG_FP64,
    load,
)
