"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds graph generators and hyperparameter draws only.  It holds
none of the embedding method's arithmetic: no sampling, aggregation, logarithm,
factorisation or propagation.  Every function is a pure function of its seed.
"""
from .graphs import (Graph, sbm, chung_lu, workload, dirichlet_s,
                     trial_vectors, pair_weights, relabel, WORKLOADS)
from .links import holdout_edges, corrupt_destinations

__all__ = ["Graph", "sbm", "chung_lu", "workload", "dirichlet_s",
           "trial_vectors", "pair_weights", "relabel", "WORKLOADS", "holdout_edges",
           "corrupt_destinations"]
