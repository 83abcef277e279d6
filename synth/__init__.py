"""Seeded synthetic inputs for the macroscopic cross-section lookup.

Both the CPU oracle tests and the GPU path draw their tables and queries from
here; this package computes nothing of the lookup itself.
"""
from .rng import Stream, mix64, stream_key  # noqa: F401
from .workloads import (  # noqa: F401
    BASE_SEED, N_CHANNELS, Queries, Tables, config1_tables, config1_queries,
    config2_tables, config2_queries, config3_queries, config4_queries,
    config5_requests, random_tables, random_queries, mean_nuclides,
)
