"""GPU: colour pruning (preprocessing step (i)) keeps every result bit for bit:
per-point values, localisation by input edge id, vertex localisation, time
buckets and extracted paths equal those of the full graph and the oracle."""

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


def _kept(g, colors):
    keep = np.isin(g.color, list(colors))
    return int(np.count_nonzero(keep[g.src] & keep[g.dst]))


def test_prune_random_graphs(tpm):
    rng = np.random.default_rng(91)
    for it in range(40):
        g = G.random_tiny_graph(rng, n_max=40, m_max=200, t_max=8, q_max=5)
        k = int(rng.integers(2, 7))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        extra = [int(c) for c in rng.integers(0, g.num_colors, int(rng.integers(0, 2)))]
        seed = int(rng.integers(0, 2**63))
        say(f"case prune rand{it}: n={g.n} m={g.m} k={k}")
        Gd = tpm.Graph.from_temporal(g, tile_edges=int(rng.integers(1, 64)))
        Gp = Gd.prune(set(M) | set(extra))
        st = Gp.stats()
        assert st["m"] == _kept(g, set(M) | set(extra)) and st["edge_ids"] == g.m
        pp, tot, loc = Gp.sieve(M, seed, loc=True)
        wpp, wloc = oracle.sieve(g, M, seed, loc=True)
        assert np.array_equal(pp, wpp) and np.array_equal(loc, wloc), it
        assert np.array_equal(Gp.sieve_vertex(M, seed), oracle.vertex_sieve(g, M, seed))
        t_full, b_full = oracle.time_buckets(g, M, seed)
        full = dict(zip(t_full.tolist(), b_full.tolist()))
        if st["m"]:
            t, b = Gp.time_buckets(M, seed)
            for tt, bb in zip(t.tolist(), b.tolist()):
                assert full[tt] == bb
            # times present only in the full graph carry no path
            assert all(v == 0 for tt, v in full.items() if tt not in set(t.tolist()))
        assert Gp.optimum_time(M, seed, reps=2) == oracle.optimum_time(g, M, seed, reps=2)
        r1 = Gd.extract(M, seed, max_reps=6)
        r2 = Gp.extract(M, seed, max_reps=6)
        assert r1[0] == r2[0] and list(r1[1]) == list(r2[1]) and list(r1[2]) == list(r2[2])
        if r2[0] == tpm.TPM_OK:
            assert pyref.check_path(g, M, r2[1], r2[2])
        Gp.close()
        Gd.close()


def test_prune_hub_graph_and_empty(tpm):
    g = G.chung_lu_graph(20000, 400000, 2.5, 300, 8, 92)
    Gd = tpm.Graph.from_temporal(g)
    for M in ([0, 1, 2, 0, 1, 2, 3], [5, 5, 6]):
        say(f"case prune hubs M={M}")
        Gp = Gd.prune(M)
        assert Gp.stats()["m"] == _kept(g, M)
        pp, _ = Gp.sieve(M, 17)
        assert np.array_equal(pp, oracle.sieve(g, M, 17))
        assert np.array_equal(pp, Gd.sieve(M, 17)[0])
        Gp.close()
    # a colour no vertex has: nothing kept
    g2 = G.uniform_graph(100, 1000, 20, 3, 4)
    g2.color[:] = np.minimum(g2.color, 1)
    Gd2 = tpm.Graph.from_temporal(g2)
    Gp = Gd2.prune([2])
    assert Gp.stats()["m"] == 0
    assert Gp.sieve([2, 2], 3)[1] == 0
    Gp.close()
    Gd2.close()
    with pytest.raises(tpm.TpmError):
        Gd.prune([8])  # colour out of range
    Gd.close()


def test_ec_path_motif_by_time_pruning(tpm):
    """EC-PATH-MOTIF: the plain sieve on the edges at the prescribed times equals the
    paper's EC recursion evaluated by the reference, per point."""
    rng = np.random.default_rng(93)
    checked = 0
    for it in range(40):
        g = G.random_tiny_graph(rng, n_max=30, m_max=150, t_max=7, q_max=4)
        k = int(rng.integers(2, 6))
        if g.m == 0 or len(np.unique(g.tau)) < k - 1:
            continue
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        times = sorted(int(t) for t in rng.choice(np.unique(g.tau), k - 1, replace=False))
        say(f"case ec{it}: k={k} times={times}")
        Gd = tpm.Graph.from_temporal(g)
        Gp = Gd.prune(times=times)
        assert Gp.stats()["m"] == int(np.isin(g.tau, times).sum())
        pp, _ = Gp.sieve(M, 60 + it)
        assert np.array_equal(pp, pyref.ec_per_point(g, M, 60 + it, times)), it
        Gc = Gd.prune(colors=set(M), times=times)  # both filters
        assert np.array_equal(Gc.sieve(M, 60 + it)[0], pp)
        Gc.close()
        Gp.close()
        Gd.close()
        checked += 1
    assert checked > 15


def test_pruned_tuning_in_sieve_and_batch(tpm):
    """tuning.prune: sieves and batches run each query on its colour subgraph (memory
    reused across calls) with the same results; wildcard queries use the whole graph."""
    g = G.chung_lu_graph(5000, 80000, 2.5, 60, 6, 94)
    rng = np.random.default_rng(95)
    Gd = tpm.Graph.from_temporal(g)
    for it in range(8):
        M = [int(c) for c in rng.integers(-1 if it % 4 == 3 else 0, 6, int(rng.integers(2, 10)))]
        say(f"case pruned tuning {it}: M={M}")
        pp, tot, loc = Gd.sieve(M, 11 + it, loc=True, prune=True)
        wpp, wloc = oracle.sieve(g, M, 11 + it, loc=True)
        assert np.array_equal(pp, wpp) and np.array_equal(loc, wloc)
    qs = [{"multiset": [int(c) for c in rng.integers(0, 6, int(rng.integers(2, 9)))],
           "seed": int(rng.integers(0, 2**62)), "want_path": 1} for _ in range(20)]
    res = Gd.batch(qs, prune=True)
    for q, r in zip(qs, res):
        assert r["total"] == oracle.sieve_total(g, q["multiset"], q["seed"])
        if r["found"]:
            k = len(q["multiset"])
            assert r["path_status"] == tpm.TPM_OK
            assert pyref.check_path(g, q["multiset"], r["path_vertices"][:k], r["path_edges"][:k - 1])
    Gd.close()


def _host_rows(src, dst, tau, n):
    """Rows and gathers of an index, recomputed on the host: each edge (u -> v, t) reads
    the last position of u's in-list (sorted by arrival) with an earlier time; rows are
    the distinct positions read, gathers the edges that read one."""
    if src.size == 0:
        return 0, 0
    T = int(tau.max()) + 1
    keys = np.sort(dst.astype(np.int64) * T + tau)
    q = np.searchsorted(keys, src.astype(np.int64) * T + tau, side="left") - 1
    lo = np.searchsorted(keys, src.astype(np.int64) * T, side="left")
    q = np.where(q >= lo, q, -1)
    read = q[q >= 0]
    return int(np.unique(read).size), int(read.size)


@pytest.mark.parametrize("m", [991, 992, 993, 2976, 2977, 6000])
def test_prune_record_boundaries(tpm, m):
    """Kept edges are flagged in records of 992 positions and read positions and rows
    are ranked through them: edge counts around record boundaries, every colour kept,
    one colour kept; rows and gathers of the full graph and of each subgraph equal a
    host recount, and the sieve equals the oracle."""
    g = G.uniform_graph(60, m, 12, 3, 700 + m)
    Gd = tpm.Graph.from_temporal(g, tile_edges=64)
    st = Gd.stats()
    assert (st["rows"], st["gathers"]) == _host_rows(g.src, g.dst, g.tau, g.n)
    for colors in ([0, 1, 2], [1], [0, 2]):
        say(f"case prune records m={m} colours={colors}")
        keep = np.isin(g.color, colors)
        e = keep[g.src] & keep[g.dst]
        Gp = Gd.prune(colors)
        sp = Gp.stats()
        assert sp["m"] == int(e.sum())
        assert (sp["rows"], sp["gathers"]) == _host_rows(g.src[e], g.dst[e], g.tau[e], g.n)
        M = [colors[0], colors[-1], colors[0]]
        pp, _ = Gp.sieve(M, 5 + m)
        assert np.array_equal(pp, oracle.sieve(g, M, 5 + m))
        Gp.close()
    Gd.close()
