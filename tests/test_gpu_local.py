"""GPU: localised outputs (vertex-localised sieve, per-timestamp buckets, optimum
timestamp) through the C ABI against the oracle, byte for byte."""

import sys

import numpy as np
import pytest

import oracle
from oracle import pyref
from synth import graphs as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tpm():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2001_07158_amd import tpm as _tpm
    return _tpm


def test_vertex_and_time_random_small(tpm):
    rng = np.random.default_rng(71)
    for it in range(60):
        g = G.random_tiny_graph(rng, n_max=40, m_max=200, t_max=8, q_max=4)
        k = int(rng.integers(2, 7))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        seed = int(rng.integers(0, 2**63))
        mask = None if it % 3 else (rng.random(g.n) < 0.8).astype(np.uint8)
        say(f"case local rand{it}: n={g.n} m={g.m} k={k}")
        Gd = tpm.Graph.from_temporal(g, tile_edges=int(rng.integers(1, 64)))
        q = Gd.sieve_vertex(M, seed, mask=mask)
        assert np.array_equal(q, oracle.vertex_sieve(g, M, seed, mask=mask)), it
        if g.m:
            times, b = Gd.time_buckets(M, seed)
            wt, wb = oracle.time_buckets(g, M, seed)
            assert np.array_equal(times, wt) and np.array_equal(b, wb), it
        assert Gd.optimum_time(M, seed, reps=2) == oracle.optimum_time(g, M, seed, reps=2)
        Gd.close()


def test_optimum_time_against_exhaustive_search(tpm):
    rng = np.random.default_rng(72)
    exact = total = 0
    for it in range(40):
        g = G.random_tiny_graph(rng, n_max=10, m_max=30, t_max=8)
        k = int(rng.integers(2, 5))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        best = pyref.brute_optimum_time(g, M)
        Gd = tpm.Graph.from_temporal(g)
        got = Gd.optimum_time(M, 500 + it, reps=3)
        Gd.close()
        if best < 0:
            assert got == -1
            continue
        total += 1
        assert got == -1 or got >= best
        exact += got == best
    assert total > 5 and exact >= total - 2


def test_local_hub_graph_and_stats(tpm):
    g = G.chung_lu_graph(20000, 400000, 2.5, 300, 4, 73)
    M = [0, 1, 2, 3, 0, 1]
    Gd = tpm.Graph.from_temporal(g)
    assert Gd.stats()["times"] == np.unique(g.tau).size
    for seed in (3, 4):
        say(f"case local hubs seed={seed}")
        assert np.array_equal(Gd.sieve_vertex(M, seed), oracle.vertex_sieve(g, M, seed))
        t, b = Gd.time_buckets(M, seed)
        wt, wb = oracle.time_buckets(g, M, seed)
        assert np.array_equal(t, wt) and np.array_equal(b, wb)
    assert Gd.optimum_time(M, 3, reps=2) == oracle.optimum_time(g, M, 3, reps=2)
    Gd.close()


def test_local_degenerate(tpm):
    g = G.TemporalGraph(4, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                        np.array([0, 1, 0, 1], np.int32), 2)
    Gd = tpm.Graph.from_temporal(g)
    assert not Gd.sieve_vertex([0, 1], 3).any()
    t, b = Gd.time_buckets([0, 1], 3)
    assert t.size == 0 and b.size == 0
    assert Gd.optimum_time([0, 1], 3) == -1
    with pytest.raises(tpm.TpmError):
        Gd.sieve_vertex([0], 3)  # k = 1 has no edges to localise
    Gd.close()


@pytest.mark.parametrize("method", [0, 1, 2])
def test_extract_optimum_against_exhaustive_search(tpm, method):
    """An optimum solution: the optimum time, then a path on the subgraph of edges that
    arrive by it; the path is valid and finishes by that time, which is never below the
    exhaustive-search optimum and equals it on nearly every instance."""
    rng = np.random.default_rng(74 + method)
    exact = total = 0
    for it in range(30):
        g = G.random_tiny_graph(rng, n_max=10, m_max=30, t_max=8)
        k = int(rng.integers(2, 5))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        best = pyref.brute_optimum_time(g, M)
        say(f"case optimum-extract m{method} {it}: n={g.n} m={g.m} M={M} best={best}")
        Gd = tpm.Graph.from_temporal(g)
        rc, t, verts, edges = Gd.extract_optimum(M, 700 + it, reps=4, method=method)
        Gd.close()
        if best < 0:
            assert rc == tpm.TPM_NOTFOUND and t == -1
            continue
        total += 1
        if rc == tpm.TPM_OK:
            assert pyref.check_path(g, M, verts, edges)
            assert t >= best and int(g.tau[edges[-1]]) <= t
            exact += int(g.tau[edges[-1]]) == best
    assert total > 5 and exact >= total - 3
