"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Holds none of the box code's arithmetic: it draws Gaussian-bump sources, builds adaptive
2:1-balanced quadtrees that resolve them, and samples the source at leaf nodes.
"""
from .gen import (  # noqa: F401
    Workload,
    config1,
    config2,
    config3,
    config4,
    config5,
    uniform_tree,
    random_small_tree,
    sample_gaussians,
)
