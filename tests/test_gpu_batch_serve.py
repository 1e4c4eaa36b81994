"""GPU: the batched form and the serving loop give, for every query, exactly the
value of the same query run alone (and of the CPU oracle)."""

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


@pytest.fixture(scope="module")
def graph():
    return G.chung_lu_graph(3000, 40000, 2.5, 60, 5, 21)


def _queries(rng, n, q, kmin=1, kmax=11):
    out = []
    for _ in range(n):
        k = int(rng.integers(kmin, kmax + 1))
        out.append({"multiset": [int(c) for c in rng.integers(0, q, k)],
                    "seed": int(rng.integers(0, 2**62))})
    return out


@pytest.mark.parametrize("chunk", [0, 256, 512])
def test_batch_totals_match_oracle(tpm, graph, chunk):
    rng = np.random.default_rng(100 + chunk)
    qs = _queries(rng, 60, graph.num_colors)
    say(f"case batch chunk={chunk}: {len(qs)} queries")
    Gd = tpm.Graph.from_temporal(graph)
    res = Gd.batch(qs, chunk=chunk)
    for q, r in zip(qs, res):
        want = oracle.sieve_total(graph, q["multiset"], q["seed"])
        assert r["total"] == want, (q, r["total"], want)
        assert r["found"] == (want != 0)
    Gd.close()


@pytest.mark.parametrize("chunk", [0, 256])
def test_batch_graph_replay_matches_plain_and_oracle(tpm, graph, chunk):
    """Passes of one row shape replay one captured HIP graph; eager work (x rows,
    clears, reads with a synchronisation) runs between the replays.  Every pass is
    checked against plain launches and the oracle."""
    rng = np.random.default_rng(300 + chunk)
    # 37 queries of k = 6 (several passes of one shape, then a shorter last pass),
    # plus mixed sizes
    qs = [{"multiset": [int(c) for c in rng.integers(0, graph.num_colors, 6)],
           "seed": int(rng.integers(0, 2**62))} for _ in range(37)]
    qs += _queries(rng, 20, graph.num_colors, 2, 9)
    say(f"case batch graph chunk={chunk}: {len(qs)} queries")
    Gd = tpm.Graph.from_temporal(graph)
    plain = Gd.batch(qs, chunk=chunk)
    for rep in range(2):
        res = Gd.batch(qs, chunk=chunk, use_graph=True)
        for i, (q, a, b) in enumerate(zip(qs, plain, res)):
            assert a["total"] == b["total"], (rep, i, q)
    for q, r in zip(qs, plain):
        assert r["total"] == oracle.sieve_total(graph, q["multiset"], q["seed"])
    Gd.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_fingerprint_plans(tpm, graph, use_graph):
    """A step finds y either from a table of <= 8 (seed, level) groups hashed once
    per 64 positions, or from a shared inner hash (one level, many seeds), or per
    lane: rows of 6 (table), 12 and 40 (shared inner) queries of one size."""
    rng = np.random.default_rng(55)
    qs = []
    for k, cnt in ((6, 6), (5, 12), (4, 40), (7, 3)):
        qs += [{"multiset": [int(c) for c in rng.integers(0, graph.num_colors, k)],
                "seed": int(rng.integers(0, 2**62))} for _ in range(cnt)]
    say(f"case fingerprint plans graph={use_graph}")
    Gd = tpm.Graph.from_temporal(graph)
    res = Gd.batch(qs, use_graph=use_graph)
    for q, r in zip(qs, res):
        assert r["total"] == oracle.sieve_total(graph, q["multiset"], q["seed"]), q
    Gd.close()


def test_batch_with_paths(tpm):
    g = G.uniform_graph(300, 3000, 40, 3, 5)
    rng = np.random.default_rng(2)
    qs = _queries(rng, 20, 3, 2, 5)
    for q in qs:
        q["want_path"] = 1
    Gd = tpm.Graph.from_temporal(g)
    res = Gd.batch(qs)
    for q, r in zip(qs, res):
        if r["found"]:
            k = len(q["multiset"])
            assert r["path_status"] == tpm.TPM_OK
            assert pyref.check_path(g, q["multiset"], r["path_vertices"][:k], r["path_edges"][:k - 1])
    Gd.close()


@pytest.mark.parametrize("lanes", [64, 24])
def test_server_matches_alone(tpm, graph, lanes):
    rng = np.random.default_rng(7 + lanes)
    qs = _queries(rng, 40, graph.num_colors, 1, 11)
    say(f"case server lanes={lanes}")
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, max_lanes=lanes)
    tickets = {}
    for i, q in enumerate(qs):
        tickets[srv.submit(q["multiset"], q["seed"])] = i
    got = srv.drain(len(qs), timeout_s=300)
    srv.close()
    assert len(got) == len(qs)
    for r in got:
        q = qs[tickets[r["ticket"]]]
        _, alone = Gd.sieve(q["multiset"], q["seed"])
        assert r["total"] == alone
        assert r["t_submit_ms"] <= r["t_start_ms"] <= r["t_done_ms"]
    Gd.close()


def test_server_alone_vs_mix_and_extraction(tpm):
    g = G.uniform_graph(400, 4000, 50, 3, 9)
    Gd = tpm.Graph.from_temporal(g)
    probe = {"multiset": [0, 1, 2, 0], "seed": 4242}
    srv = tpm.Server(Gd, extract_paths=1)
    srv.submit(probe["multiset"], probe["seed"])
    alone = srv.drain(1)[0]
    rng = np.random.default_rng(3)
    mix = _queries(rng, 25, 3, 2, 8)
    t_probe = None
    for i, q in enumerate(mix):
        t = srv.submit(q["multiset"], q["seed"])
        if i == 12:
            t_probe = srv.submit(probe["multiset"], probe["seed"])
    got = srv.drain(len(mix) + 1)
    srv.close()
    mixed = [r for r in got if r["ticket"] == t_probe][0]
    assert mixed["total"] == alone["total"]
    assert mixed["found"] == alone["found"]
    for r in got + [alone]:
        if r["found"]:
            assert r["path_status"] == tpm.TPM_OK
    if alone["found"]:
        assert pyref.check_path(g, probe["multiset"], alone["path_vertices"][:4], alone["path_edges"][:3])
    Gd.close()


def test_pruned_server_matches_alone(tpm, graph):
    """Serving with per-request colour pruning: same totals as the full graph and the
    oracle, and extracted paths check out."""
    rng = np.random.default_rng(61)
    qs = _queries(rng, 25, graph.num_colors, 1, 9)
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, prune_queries=1, extract_paths=1)
    tickets = [srv.submit(q["multiset"], q["seed"]) for q in qs]
    got = {r["ticket"]: r for r in srv.drain(len(qs), timeout_s=300)}
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(qs) and st["steps"] == len(qs)
    assert st["prune_ms"] > 0 and st["sieve_ms"] > 0 and st["row_points"] == 0
    for t, q in zip(tickets, qs):
        r = got[t]
        want = oracle.sieve_total(graph, q["multiset"], q["seed"])
        assert r["total"] == want, q
        if r["found"] and len(q["multiset"]) >= 2:
            assert r["path_status"] == tpm.TPM_OK
            k = len(q["multiset"])
            assert pyref.check_path(graph, q["multiset"], r["path_vertices"][:k],
                                    r["path_edges"][:k - 1])
    Gd.close()
