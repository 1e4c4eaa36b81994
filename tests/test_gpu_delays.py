"""GPU: the variant with transition times (per edge) and delays (per vertex), section
"Path motif problem with delays", against the oracle and exhaustive search."""

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


def _graph(tpm, g, tr, dl, **kw):
    return tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, transit=tr, delay=dl, **kw)


def test_delays_random_small(tpm):
    rng = np.random.default_rng(121)
    for it in range(60):
        g = G.random_tiny_graph(rng, n_max=40, m_max=200, t_max=8, q_max=4)
        tr = rng.integers(0, 3, g.m).astype(np.int32) if it % 3 else None
        dl = rng.integers(0, 3, g.n).astype(np.int32) if it % 4 else None
        k = int(rng.integers(2, 7))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        seed = int(rng.integers(0, 2**63))
        say(f"case delays rand{it}: n={g.n} m={g.m} k={k} transit={tr is not None} delay={dl is not None}")
        Gd = _graph(tpm, g, tr, dl, tile_edges=int(rng.integers(1, 64)))
        pp, tot, loc = Gd.sieve(M, seed, loc=True)
        wpp, wloc = oracle.sieve(g, M, seed, loc=True, transit=tr, delay=dl)
        assert np.array_equal(pp, wpp) and np.array_equal(loc, wloc), it
        assert np.array_equal(Gd.sieve_vertex(M, seed),
                              oracle.vertex_sieve(g, M, seed, transit=tr, delay=dl))
        if g.m:
            t, b = Gd.time_buckets(M, seed)
            wt, wb = oracle.time_buckets(g, M, seed, transit=tr, delay=dl)
            assert np.array_equal(t, wt) and np.array_equal(b, wb), it
        Gp = Gd.prune(set(M))
        assert np.array_equal(Gp.sieve(M, seed)[0], wpp)
        Gp.close()
        Gd.close()


def test_delays_extraction_and_optimum(tpm):
    rng = np.random.default_rng(122)
    yes = no = 0
    for it in range(50):
        g = G.random_tiny_graph(rng, n_max=12, m_max=40, t_max=6, q_max=3)
        tr = rng.integers(0, 2, g.m).astype(np.int32)
        dl = rng.integers(0, 3, g.n).astype(np.int32)
        k = int(rng.integers(2, 5))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        exists = pyref.has_matching_path(g, M, tr, dl)
        Gd = _graph(tpm, g, tr, dl)
        rc, verts, edges = Gd.extract(M, 900 + it, max_reps=12)
        if exists:
            yes += 1
            assert rc == tpm.TPM_OK, it
            assert pyref.check_path(g, M, verts, edges, tr, dl)
        else:
            no += 1
            assert rc == tpm.TPM_NOTFOUND
        assert Gd.optimum_time(M, 5 + it, reps=2) == oracle.optimum_time(g, M, 5 + it, reps=2,
                                                                       transit=tr, delay=dl)
        Gd.close()
    assert yes > 5 and no > 5


def test_delays_defaults_equal_plain_on_hub_graph(tpm):
    g = G.chung_lu_graph(3000, 60000, 2.5, 50, 3, 123)
    M = [0, 1, 2, 0, 1, 2]
    plain = tpm.Graph.from_temporal(g)
    same = _graph(tpm, g, np.zeros(g.m, np.int32), np.ones(g.n, np.int32))
    assert np.array_equal(plain.sieve(M, 4)[0], same.sieve(M, 4)[0])
    rng = np.random.default_rng(3)
    tr = rng.integers(0, 4, g.m).astype(np.int32)
    dl = rng.integers(0, 3, g.n).astype(np.int32)
    for T in (16, 1024):
        say(f"case delays hubs T={T}")
        Gd = _graph(tpm, g, tr, dl, tile_edges=T)
        assert np.array_equal(Gd.sieve(M, 4)[0], oracle.sieve(g, M, 4, transit=tr, delay=dl))
        Gd.close()
    plain.close()
    same.close()
