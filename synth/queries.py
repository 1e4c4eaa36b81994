"""Query multisets and seed conventions."""

from __future__ import annotations

import numpy as np

BASE_SEED = 200107158


def config_seed(config_index: int, query_index: int = 0) -> int:
    """Graph seed = BASE + config index; query q of that config adds 1000*q."""
    return BASE_SEED + config_index + 1000 * query_index


def random_multiset(rng: np.random.Generator, q: int, k: int) -> np.ndarray:
    """k colours drawn i.i.d. uniformly from [0, q) (a multiset, repetition allowed)."""
    return np.sort(rng.integers(0, q, k)).astype(np.int32)
