"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This package draws times and observations only.  It holds none of the
inference arithmetic (no precision blocks, no reduction, no likelihood); both
the oracle and the device path receive its arrays as plain inputs.
"""
from .generate import (  # noqa: F401
    KIND_MATERN12,
    KIND_MATERN32,
    KIND_MATERN52,
    KIND_MATERN72,
    KIND_PERIODIC,
    KIND_QUASIPERIODIC,
    KIND_SQEXP,
    Workload,
    make_batch,
    make_config,
    make_series,
    n_hyper,
    state_dim,
)
