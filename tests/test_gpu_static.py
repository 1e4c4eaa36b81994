"""GPU: the static vertex-localised sieve of preprocessing step (ii) (tpm_static_sieve)
and the subgraph it keeps (tpm_graph_prune_static), against the oracle."""

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


def test_static_random_small(tpm):
    rng = np.random.default_rng(181)
    for it in range(50):
        g = G.random_tiny_graph(rng, n_max=40, m_max=300, t_max=8, q_max=4)
        k = int(rng.integers(1, 8))
        M = [int(c) for c in rng.integers(-1 if it % 5 == 0 else 0, g.num_colors, k)]
        seed = int(rng.integers(0, 2**63))
        say(f"case static rand{it}: n={g.n} m={g.m} M={M}")
        Gd = tpm.Graph.from_temporal(g)
        assert np.array_equal(Gd.static_sieve(M, seed), oracle.static_sieve(g, M, seed)), it
        Gd.close()


@pytest.mark.parametrize("k", [2, 4, 6, 8, 9, 10])
def test_static_chung_lu(tpm, k):
    """Rows of 16..1024 points (one to four dwords a lane), hubs whose lists span many
    tiles (atomic combination), colour filtering."""
    g = G.chung_lu_graph(20000, 300000, 2.1, 50, 6, 182 + k)
    M = [int(c) for c in np.random.default_rng(k).integers(0, 6, k)]
    say(f"case static chung-lu k={k} M={M}")
    Gd = tpm.Graph.from_temporal(g)
    s = Gd.static_sieve(M, 1234 + k)
    assert np.array_equal(s, oracle.static_sieve(g, M, 1234 + k))
    Gd.close()


def test_static_hub_and_empty(tpm):
    n = 600
    src = np.concatenate([np.arange(1, n), np.zeros(n - 1)]).astype(np.int32)
    dst = np.concatenate([np.zeros(n - 1), np.arange(1, n)]).astype(np.int32)
    tau = np.arange(1, 2 * n - 1, dtype=np.int32)
    color = (np.arange(n) % 3).astype(np.int32)
    g = G.TemporalGraph(n, src, dst, tau, color, 3)
    Gd = tpm.Graph.from_temporal(g)
    for M in ([0, 1, 2], [0, 0, 1], [1, 2], [0, 1, 2, 0]):
        say(f"case static hub M={M}")
        assert np.array_equal(Gd.static_sieve(M, 5), oracle.static_sieve(g, M, 5))
    Gd.close()
    e = G.TemporalGraph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                        np.zeros(5, np.int32), 2)
    Ge = tpm.Graph.from_temporal(e)
    assert not Ge.static_sieve([0, 1], 3).any()
    assert np.array_equal(Ge.static_sieve([0], 3), oracle.static_sieve(e, [0], 3))
    Gp = Ge.prune_static([0, 1], 3)
    assert Gp.stats()["m"] == 0
    Gp.close()
    Ge.close()


def test_prune_static_matches_oracle_subgraph(tpm):
    """The kept subgraph is the one the oracle's static sieves give (vertices with a
    nonzero value for one of the seeds), checked through its per-point values; on tiny
    graphs whose matches it keeps, the sieve total is the full graph's."""
    rng = np.random.default_rng(183)
    for it in range(30):
        g = G.random_tiny_graph(rng, n_max=30, m_max=200, t_max=8, q_max=4)
        k = int(rng.integers(2, 6))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        seed, reps = int(rng.integers(0, 2**62)), int(rng.integers(1, 4))
        say(f"case prune-static {it}: n={g.n} m={g.m} M={M} reps={reps}")
        keep = np.zeros(g.n, dtype=bool)
        for r in range(reps):
            keep |= oracle.static_sieve(g, M, (seed + r * 0x9E3779B97F4A7C15) % 2**64) != 0
        em = (keep[g.src] & keep[g.dst]).astype(np.uint8)
        Gd = tpm.Graph.from_temporal(g)
        Gp = Gd.prune_static(M, seed, reps)
        assert Gp.stats()["m"] == int(em.sum())
        pp, tot = Gp.sieve(M, 77 + it)
        assert np.array_equal(pp, oracle.sieve(g, M, 77 + it, emask=em)), it
        if g.m <= 60:
            on_path = set()
            for verts, _ in pyref.temporal_walks(g, k):
                if len(set(verts)) == k and pyref.colours_match([int(g.color[u]) for u in verts], M):
                    on_path |= set(verts)
            if on_path <= set(np.nonzero(keep)[0].tolist()):
                assert tot == Gd.sieve(M, 77 + it)[1]
        Gp.close()
        Gd.close()
