"""GPU: VC-PATH-MOTIF (colours in a prescribed order) through the layered graph,
against the oracle's ordered-colour recursion and exhaustive search."""

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


def test_vc_random_small(tpm):
    rng = np.random.default_rng(131)
    for it in range(60):
        g = G.random_tiny_graph(rng, n_max=40, m_max=200, t_max=8, q_max=4)
        k = int(rng.integers(1, 7))
        C = [int(c) for c in rng.integers(0, g.num_colors, k)]
        tr = rng.integers(0, 2, g.m).astype(np.int32) if it % 3 == 0 else None
        dl = rng.integers(0, 3, g.n).astype(np.int32) if it % 3 == 0 else None
        seed = int(rng.integers(0, 2**63))
        say(f"case vc rand{it}: n={g.n} m={g.m} C={C}")
        Gd = tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, transit=tr, delay=dl)
        Gl = Gd.layer(C)
        ids = Gl.vertex_ids()
        assert all(int(g.color[u]) in C for u in ids) or Gl.stats()["m"] == 0
        pp, tot = Gl.sieve(C, seed)
        assert np.array_equal(pp, oracle.vc_sieve(g, C, seed, transit=tr, delay=dl)), it
        Gl.close()
        Gd.close()


def test_vc_extraction_against_exhaustive_search(tpm):
    rng = np.random.default_rng(132)
    yes = no = 0
    for it in range(50):
        g = G.random_tiny_graph(rng, n_max=12, m_max=40, t_max=6, q_max=3)
        k = int(rng.integers(2, 5))
        C = [int(c) for c in rng.integers(0, g.num_colors, k)]
        exists = pyref.has_vc_path(g, C)
        Gd = tpm.Graph.from_temporal(g)
        Gl = Gd.layer(C)
        rc, verts, edges = Gl.extract(C, 77 + it, max_reps=12)
        rc2, v2, e2, _ = Gl.extract_ex(C, 77 + it, max_reps=12, method=2)
        assert rc2 == rc, it
        if exists:
            yes += 1
            assert rc == tpm.TPM_OK, it
            assert pyref.check_path(g, C, verts, edges)
            assert [int(g.color[v]) for v in verts] == C  # the order itself
            assert pyref.check_path(g, C, v2, e2)
            assert [int(g.color[v]) for v in v2] == C
        else:
            no += 1
            assert rc == tpm.TPM_NOTFOUND
        Gl.close()
        Gd.close()
    assert yes > 5 and no > 5


def test_vc_hub_graph_and_degenerate(tpm):
    g = G.chung_lu_graph(20000, 400000, 2.5, 300, 4, 133)
    Gd = tpm.Graph.from_temporal(g)
    for C in ([0, 1, 2, 3, 0, 1], [2, 2, 2], [3]):
        say(f"case vc hubs C={C}")
        Gl = Gd.layer(C)
        assert np.array_equal(Gl.sieve(C, 9)[0], oracle.vc_sieve(g, C, 9))
        Gl.close()
    Gd.close()
    g2 = G.uniform_graph(50, 300, 10, 3, 6)
    g2.color[:] = np.minimum(g2.color, 1)  # colour 2 unused
    Gd2 = tpm.Graph.from_temporal(g2)
    Gl = Gd2.layer([2, 0])
    assert Gl.stats()["m"] == 0 and Gl.sieve([2, 0], 3)[1] == 0
    Gl.close()
    Gd2.close()
