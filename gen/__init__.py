"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module draws random inputs only: factor-model returns, sketch matrices,
target returns and random test vectors.  It holds none of the solver's
arithmetic (no centering, no covariance, no projection, no gradient).
Both the oracle and the HIP path read what it returns as plain data.
"""
from .factor_model import (
    FactorModelSpec,
    SPECS,
    returns_TxN,
    target_return,
    frontier_targets_from_mv,
    gaussian_sketch,
    countsketch,
    random_vector,
    heldout_returns_TxN,
)

__all__ = [
    "FactorModelSpec",
    "SPECS",
    "returns_TxN",
    "target_return",
    "frontier_targets_from_mv",
    "gaussian_sketch",
    "countsketch",
    "random_vector",
    "heldout_returns_TxN",
]
