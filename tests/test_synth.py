"""CPU: the seeded input generators produce the shapes and distributions the workloads
state (ranges, no self-loops, determinism, the power-law weights of the Chung-Lu model,
exact stub counts of the configuration model, order-preserving time relabelling)."""

import numpy as np
import pytest

from synth import graphs as G
from synth.configs import CONFIGS, make_config_graph, make_config_query


def _same(a, b):
    return (a.n == b.n and a.num_colors == b.num_colors and np.array_equal(a.src, b.src)
            and np.array_equal(a.dst, b.dst) and np.array_equal(a.tau, b.tau)
            and np.array_equal(a.color, b.color))


def _ranges(g, t):
    assert g.src.dtype == g.dst.dtype == g.tau.dtype == g.color.dtype == np.int32
    assert g.src.min() >= 0 and g.src.max() < g.n
    assert g.dst.min() >= 0 and g.dst.max() < g.n
    assert g.tau.min() >= 1 and g.tau.max() <= t
    assert g.color.min() >= 0 and g.color.max() < g.num_colors


def test_uniform_graph():
    g = G.uniform_graph(500, 20000, 50, 4, 1)
    _ranges(g, 50)
    assert g.m == 20000 and not np.any(g.src == g.dst)
    assert _same(g, G.uniform_graph(500, 20000, 50, 4, 1))
    assert not _same(g, G.uniform_graph(500, 20000, 50, 4, 2))
    # every timestamp and colour value occurs, none far from its expected share
    assert np.bincount(g.tau, minlength=51)[1:].min() > 0.6 * 20000 / 50
    assert np.bincount(g.color, minlength=4).min() > 0.7 * 500 / 4
    loops = G.uniform_graph(3, 3000, 5, 2, 4, self_loops=True)
    assert np.any(loops.src == loops.dst)


def test_alias_sampler_frequencies():
    """Walker's alias method draws index i with probability w_i / sum(w)."""
    rng = np.random.default_rng(5)
    w = np.array([1.0, 2.0, 3.0, 4.0, 0.5, 9.5])
    draw = G._alias_sampler(rng, w)
    x = draw(2_000_000)
    f = np.bincount(x, minlength=w.size) / x.size
    assert np.allclose(f, w / w.sum(), atol=2e-3)


def test_chung_lu_power_law():
    n, m, beta = 10_000, 200_000, 2.5
    g = G.chung_lu_graph(n, m, beta, 100, 8, 9)
    _ranges(g, 100)
    assert g.m == m and not np.any(g.src == g.dst)
    assert _same(g, G.chung_lu_graph(n, m, beta, 100, 8, 9))
    # the heaviest vertex draws about m * w_max / sum(w) of the edge ends
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (beta - 1.0))
    top = m * w[0] / w.sum()
    for deg in (np.bincount(g.dst, minlength=n), np.bincount(g.src, minlength=n)):
        assert 0.8 * top < deg.max() < 1.2 * top
        assert deg.max() > 20 * deg.mean()  # heavy tail
        # ranked degrees follow the ranked weights (top 20 within 25 %)
        assert np.allclose(np.sort(deg)[::-1][:20], m * w[:20] / w.sum(), rtol=0.25)


def test_regular_graph_stub_counts():
    g = G.regular_graph(1000, 6, 30, 5, 3)
    _ranges(g, 30)
    assert g.m == 1000 * 6 // 2
    ends = np.bincount(np.concatenate([g.src, g.dst]), minlength=1000)
    assert np.all(ends == 6)  # each vertex has exactly d stubs
    with pytest.raises(ValueError):
        G.regular_graph(5, 3, 10, 2, 1)


def test_relabel_keeps_order():
    rng = np.random.default_rng(8)
    g = G.uniform_graph(50, 500, 20, 3, 6)
    h = G.relabel_timestamps(g, rng)
    # a strictly increasing map: equal stays equal, smaller stays smaller
    a, b = g.tau[:, None], g.tau[None, :]
    assert np.array_equal(a < b, h.tau[:, None] < h.tau[None, :])
    assert np.array_equal(a == b, h.tau[:, None] == h.tau[None, :])
    assert h.tau.min() >= 1


def test_hardness_construction():
    edges = [(0, 1), (1, 2), (2, 3)]
    g = G.static_to_temporal_layers(4, edges, 4)
    assert g.m == 2 * 3 * len(edges)
    for a, b in edges:
        for j in range(1, 4):
            assert np.any((g.src == a) & (g.dst == b) & (g.tau == j))
            assert np.any((g.src == b) & (g.dst == a) & (g.tau == j))


def test_workload_configs():
    """The workload table's sizes, and its small case built exactly as stated."""
    assert CONFIGS["k10"]["m"] == 100_000_000 and CONFIGS["k10"]["k"] == 10
    assert CONFIGS["serving"]["m"] == 1_000_000_000
    g = make_config_graph("tiny")
    c = CONFIGS["tiny"]
    assert (g.n, g.m, g.num_colors) == (c["n"], c["m"], c["q"])
    _ranges(g, c["t"])
    assert list(make_config_query("tiny")) == c["multiset"]
    q = make_config_query("batched", 3)
    assert CONFIGS["batched"]["k_lo"] <= len(q) <= CONFIGS["batched"]["k_hi"]
    assert q.min() >= 0 and q.max() < CONFIGS["batched"]["q"]
    assert np.array_equal(q, make_config_query("batched", 3))
