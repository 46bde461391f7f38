"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This package builds inputs only: random geometric graphs, component-state
probabilities, hazard fields and reference-state rows.  It holds none of the
RSR method's arithmetic (no sampling of component states, no dominance test,
no system-function evaluation on sampled states, no estimator), so that the
oracle and the GPU library can both consume its output without sharing code.

All randomness comes from numpy's PCG64 generator with explicit seeds.
"""
from .graphs import rgg, st_farthest_pair, st_degree_rule  # noqa: F401
from .refs import (  # noqa: F401
    all_min_paths, all_min_cuts, sample_paths, sample_cuts, paths_to_upper, cuts_to_lower,
    bernoulli_rows,
)
from . import configs  # noqa: F401
