"""Named synthetic workloads (sizes, distributions, seeds).

Each workload is a seeded synthetic stand-in for the paper's graph workloads
(random regular / power-law graphs with uniform timestamps and uniform random
vertex colours, as in its experimental-setup section).  The directed Chung-Lu
model replaces the paper's own configuration-model generator.
"""

from __future__ import annotations

import numpy as np

from .graphs import TemporalGraph, chung_lu_graph, uniform_graph
from .queries import config_seed, random_multiset

CONFIGS = {
    # directed uniform graph, 4 colours, query {c1,c1,c2,c3}
    "tiny": dict(index=0, kind="uniform", n=1_000, m=10_000, t=100, q=4, k=4,
                 multiset=[0, 0, 1, 2]),
    # Chung-Lu beta=2.5, 8 colours, 5 i.i.d. colours
    "k5": dict(index=1, kind="chung_lu", n=1_000_000, m=10_000_000, beta=2.5, t=1_000, q=8, k=5),
    # Chung-Lu beta=2.5, 16 colours, 10 i.i.d. colours
    "k10": dict(index=2, kind="chung_lu", n=1_000_000, m=100_000_000, beta=2.5, t=10_000, q=16, k=10),
    # 256 queries k ~ U{3..10} over one resident graph
    "batched": dict(index=3, kind="chung_lu", n=2_000_000, m=100_000_000, beta=2.5, t=10_000, q=16,
                    nq=256, k_lo=3, k_hi=10),
    # Poisson stream against a 1e9-edge graph
    "serving": dict(index=4, kind="chung_lu", n=10_000_000, m=1_000_000_000, beta=2.5, t=100_000, q=16,
                    nq=10_000, k_lo=3, k_hi=10),
}


def make_config_graph(name: str, scale: float = 1.0) -> TemporalGraph:
    """Build the named workload's graph; `scale` < 1 shrinks n and m together
    (used only by smaller test variants, never by the bench)."""
    c = CONFIGS[name]
    n = max(2, int(round(c["n"] * scale)))
    m = max(0, int(round(c["m"] * scale)))
    seed = config_seed(c["index"])
    if c["kind"] == "uniform":
        return uniform_graph(n, m, c["t"], c["q"], seed)
    return chung_lu_graph(n, m, c["beta"], c["t"], c["q"], seed)


def make_config_query(name: str, query_index: int = 0) -> np.ndarray:
    c = CONFIGS[name]
    if "multiset" in c and query_index == 0:
        return np.array(c["multiset"], dtype=np.int32)
    rng = np.random.default_rng(config_seed(c["index"], query_index + 1))
    k = c.get("k")
    if k is None:
        k = int(rng.integers(c["k_lo"], c["k_hi"] + 1))
    return random_multiset(rng, c["q"], k)
