"""Seeded random streams for the synthetic workloads."""

import numpy as np

SEED_ROOT = 230303681

PURPOSE_INTEGRALS = 0
PURPOSE_ANGLES = 1
PURPOSE_SAMPLE = 2
PURPOSE_ARRIVALS = 3
PURPOSE_MIX = 4  # fragment shapes of the serving mix


def workload_rng(config: int, purpose: int, extra: int = 0) -> np.random.Generator:
    """PCG64 stream for (config, purpose[, extra]); extra distinguishes fragments."""
    key = [SEED_ROOT, int(config), int(purpose)]
    if extra:
        key.append(int(extra))
    return np.random.default_rng(key)
