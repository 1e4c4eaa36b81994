"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This package only draws graphs, colourings and query multisets.  It holds none of
the sieve's arithmetic (no field operations, no fingerprints, no dynamic program),
so it can serve both sides of a parity check without coupling them.
"""

from .graphs import (  # noqa: F401
    TemporalGraph,
    uniform_graph,
    chung_lu_graph,
    regular_graph,
    paper_toy_graph,
    random_tiny_graph,
    relabel_timestamps,
    append_isolated,
    static_to_temporal_layers,
)
from .queries import random_multiset, config_seed  # noqa: F401
from .configs import CONFIGS, make_config_graph, make_config_query  # noqa: F401
