"""CPU oracle for Pruned Landmark Labeling (test infrastructure only).

A plain, sequential C implementation of the paper's algorithms
(``pll_oracle.c``) behind a small ctypes wrapper.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg use it; the GPU library
never imports, links or calls anything here, and nothing here imports the
GPU library.
"""
from .oracle import (  # noqa: F401
    COUNTER_NAMES,
    DirectedIndex,
    OracleError,
    OracleIndex,
    WINF,
    WeightedIndex,
    build,
    build_directed,
    build_library,
    build_weighted,
    load_variant,
    source_text,
    paths,
    paths_weighted,
    query,
    query_directed,
    query_parts,
    query_weighted,
)
