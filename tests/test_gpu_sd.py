"""GPU: (s,d)-COLORFUL-PATH instances (tpm_graph_sd) against the oracle's own
reduction and against exhaustive search."""

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


def test_sd_random_small_against_oracle(tpm):
    """Per-point values and per-edge localisation (by input id) of the sd instance
    equal the oracle's sieve of its own reduction; paths found go s -> ... -> d."""
    rng = np.random.default_rng(171)
    for it in range(40):
        g = G.random_tiny_graph(rng, n_max=40, m_max=240, t_max=9, q_max=5)
        if g.n < 2:
            continue
        k = int(rng.integers(0, 5))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        s, d = (int(x) for x in rng.choice(g.n, 2, replace=False))
        seed = int(rng.integers(0, 2**63))
        say(f"case sd rand{it}: n={g.n} m={g.m} s={s} d={d} M={M}")
        Gd = tpm.Graph.from_temporal(g, tile_edges=int(rng.integers(1, 64)))
        Gs = Gd.sd(s, d)
        st = Gs.stats()
        assert st["num_colors"] == g.num_colors + 2 and st["n"] == g.n
        gs, em = oracle.sd_instance(g, s, d)
        assert st["m"] == int(em.sum())
        Mp = M + [g.num_colors, g.num_colors + 1]
        pp, tot, loc = Gs.sieve(Mp, seed, loc=True)
        wpp, wloc = oracle.sieve(gs, Mp, seed, emask=em, loc=True)
        assert np.array_equal(pp, wpp), it
        assert np.array_equal(loc, wloc), it
        rc, verts, edges = Gs.extract(Mp, seed, max_reps=4)
        if rc == tpm.TPM_OK:
            assert verts[0] == s and verts[-1] == d
            assert all(em[e] for e in edges)
            assert pyref.check_path(gs, Mp, verts, edges)
        Gs.close()
        Gd.close()


def test_sd_planted_colourful_path(tpm):
    """A planted s -> v1 -> ... -> vk -> d path with distinct internal colours on a
    Chung-Lu graph: decided, extracted, and the per-point values equal the oracle's."""
    g = G.chung_lu_graph(3000, 40000, 2.5, 60, 8, 172)
    rng = np.random.default_rng(5)
    k = 6
    verts = [int(v) for v in rng.choice(g.n, k + 2, replace=False)]
    color = g.color.copy()
    for i, v in enumerate(verts[1:-1]):
        color[v] = i
    times = np.arange(1, k + 2, dtype=np.int32) * 7
    src = np.concatenate([g.src, np.array(verts[:-1], dtype=np.int32)])
    dst = np.concatenate([g.dst, np.array(verts[1:], dtype=np.int32)])
    tau = np.concatenate([g.tau, times])
    h = G.TemporalGraph(g.n, src, dst, tau, color, g.num_colors)
    s, d = verts[0], verts[-1]
    M = list(range(k))
    say(f"case sd planted: n={h.n} m={h.m} s={s} d={d} k={k}")
    Gd = tpm.Graph.from_temporal(h)
    Gs = Gd.sd(s, d)
    Mp = M + [h.num_colors, h.num_colors + 1]
    gs, em = oracle.sd_instance(h, s, d)
    pp, _ = Gs.sieve(Mp, 9)
    assert np.array_equal(pp, oracle.sieve(gs, Mp, 9, emask=em))
    assert Gs.decide(Mp, 9, reps=4)
    rc, pv, pe = Gs.extract(Mp, 9, max_reps=8)
    assert rc == tpm.TPM_OK
    assert pv[0] == s and pv[-1] == d
    assert pyref.check_path(gs, Mp, pv, pe)
    Gs.close()
    Gd.close()


def test_sd_errors(tpm):
    g = G.uniform_graph(30, 100, 10, 3, 173)
    Gd = tpm.Graph.from_temporal(g)
    for s, d in ((3, 3), (-1, 2), (2, 30)):
        with pytest.raises(tpm.TpmError) as ei:
            Gd.sd(s, d)
        assert ei.value.code == tpm.TPM_EINVAL
    Gd.close()
