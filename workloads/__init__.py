"""Seeded synthetic inputs for the PC-sample attribution path.

This package only draws inputs: program structure (function, inline and loop
ranges, line ranges), a static call graph with call-instruction sites, a host
calling-context table, and PC-sample streams.  It holds none of the
attribution arithmetic; both the CPU oracle and the GPU path read what it
produces.
"""
from .gen import (  # noqa: F401
    Workload,
    config1,
    config2,
    small_config,
    tiny_random_case,
    make_samples,
    learned_intervals,
    learned_queries,
    learned_queries_gpu,
)
from .batched import batched_sizes, batched_structures, GpuSampler  # noqa: F401
