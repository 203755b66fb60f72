"""Seeded synthetic inputs shared by the oracle's tests, the GPU tests and the benchmark.

This package only *draws* inputs: graphs (stochastic block models, their perturbed
sequences, a Chung-Lu graph with planted communities, and small textbook graphs) and
Gaussian signal blocks.  It contains none of the clustering method's arithmetic: no
Laplacian, no filter, no eigencount, no k-means.  Both the FP64 oracle and the HIP
library consume what it returns, and neither side imports the other.

Seeds follow one recipe everywhere: ``base = 20170603 + 100 * config``; the graph uses
``base + 0``, feature signals ``base + 1``, eigencount probes ``base + 2``, k-means
draws ``base + 3`` and graph perturbations ``base + 4``.
"""

from .graphs import (  # noqa: F401
    Graph,
    DynamicSBM,
    block_sizes_equal,
    block_sizes_zipf,
    chung_lu,
    cycle_graph,
    disjoint_cliques,
    edges_to_graph,
    sbm,
)
from .signals import gaussian_block, seed_for  # noqa: F401
from .configs import CONFIGS, config_seed  # noqa: F401
