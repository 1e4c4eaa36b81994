"""GPU: the batched form and the serving loop give, for every query, exactly the
per-point values of the CPU oracle (byte for byte, all 2^k sieve points), alone and in
a mix; plus cancellation, deadlines and refusal of requests that cannot fit."""

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
    return G.chung_lu_graph(2000, 20000, 2.5, 60, 5, 21)


_ORACLE = {}


def want(g, q):
    """Oracle per-point values of a query (cached per graph, multiset and seed)."""
    key = (id(g), tuple(q["multiset"]), q["seed"])
    if key not in _ORACLE:
        _ORACLE[key] = oracle.sieve(g, q["multiset"], q["seed"])
    return _ORACLE[key]


def _queries(rng, n, q, kmin=1, kmax=11, wild=0.0):
    out = []
    for _ in range(n):
        k = int(rng.integers(kmin, kmax + 1))
        ms = [int(c) for c in rng.integers(0, q, k)]
        if wild and rng.random() < wild:
            ms[int(rng.integers(0, k))] = -1
        out.append({"multiset": ms, "seed": int(rng.integers(0, 2**62))})
    return out


def _check_per_point(g, qs, res):
    for i, (q, r) in enumerate(zip(qs, res)):
        w = want(g, q)
        assert r["status"] == 0, (i, q, r["status"])
        assert np.array_equal(r["per_point"], w), (i, q, np.nonzero(r["per_point"] != w)[0][:8])
        t = int(np.bitwise_xor.reduce(w))
        assert r["total"] == t and r["found"] == (t != 0), (i, q)


@pytest.mark.parametrize("chunk", [0, 256, 512])
def test_batch_per_point_matches_oracle(tpm, graph, chunk):
    """Packed rows with uneven k side by side (1..11, so queries above one row run in
    chunks), wildcards included: every per-point byte equals the oracle's."""
    rng = np.random.default_rng(100 + chunk)
    qs = _queries(rng, 60, graph.num_colors, wild=0.15)
    say(f"case batch chunk={chunk}: {len(qs)} queries")
    Gd = tpm.Graph.from_temporal(graph)
    res = Gd.batch(qs, chunk=chunk, per_point=True)
    _check_per_point(graph, qs, res)
    Gd.close()


@pytest.mark.parametrize("chunk", [0, 256])
def test_batch_graph_replay_matches_oracle(tpm, graph, chunk):
    """Row steps replayed from a captured HIP graph (lane tables uploaded before every
    replay, eager x-row work and reads with a synchronisation between replays): every
    per-point byte equals plain launches and the oracle, over two batches."""
    rng = np.random.default_rng(300 + chunk)
    qs = [{"multiset": [int(c) for c in rng.integers(0, graph.num_colors, 6)],
           "seed": int(rng.integers(0, 2**62))} for _ in range(37)]
    qs += _queries(rng, 20, graph.num_colors, 2, 9)
    say(f"case batch graph chunk={chunk}: {len(qs)} queries")
    Gd = tpm.Graph.from_temporal(graph)
    plain = Gd.batch(qs, chunk=chunk, per_point=True)
    _check_per_point(graph, qs, plain)
    for rep in range(2):
        res = Gd.batch(qs, chunk=chunk, use_graph=True, per_point=True)
        for i, (a, b) in enumerate(zip(plain, res)):
            assert np.array_equal(a["per_point"], b["per_point"]), (rep, i)
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
    res = Gd.batch(qs, use_graph=use_graph, per_point=True)
    _check_per_point(graph, qs, res)
    Gd.close()


@pytest.mark.parametrize("streams", [1, 3, 4])
def test_batch_pruned_streams_match_oracle(tpm, graph, streams):
    """Each query alone on its colour subgraph, `streams` of them at once: per-point
    bytes equal the oracle's, and a second batch reuses the graph's worker memory."""
    rng = np.random.default_rng(700 + streams)
    qs = _queries(rng, 40, graph.num_colors, 1, 10, wild=0.1)
    say(f"case pruned batch streams={streams}")
    Gd = tpm.Graph.from_temporal(graph)
    for rep in range(2):
        res = Gd.batch(qs, prune=True, streams=streams, per_point=True)
        _check_per_point(graph, qs, res)
    Gd.close()


@pytest.mark.parametrize("prune", [False, True])
def test_batch_with_paths(tpm, prune):
    g = G.uniform_graph(300, 3000, 40, 3, 5)
    rng = np.random.default_rng(2)
    qs = _queries(rng, 20, 3, 2, 5)
    for q in qs:
        q["want_path"] = 1
    Gd = tpm.Graph.from_temporal(g)
    res = Gd.batch(qs, prune=prune, per_point=True)
    _check_per_point(g, qs, res)
    for q, r in zip(qs, res):
        if r["found"]:
            k = len(q["multiset"])
            assert r["path_status"] == tpm.TPM_OK
            assert pyref.check_path(g, q["multiset"], r["path_vertices"][:k], r["path_edges"][:k - 1])
    Gd.close()


def _serve(srv, qs, per_point=True, timeout_s=300):
    tickets = [srv.submit(q["multiset"], q["seed"], per_point=per_point) for q in qs]
    got = {r["ticket"]: r for r in srv.drain(len(qs), timeout_s=timeout_s)}
    return [got[t] for t in tickets]


@pytest.mark.parametrize("lanes", [64, 24])
def test_row_server_matches_oracle(tpm, graph, lanes):
    """Row mode (continuous batching on one resident row): every streamed result
    equals the oracle per point; submission times are ordered."""
    rng = np.random.default_rng(7 + lanes)
    qs = _queries(rng, 40, graph.num_colors, 1, 11, wild=0.1)
    say(f"case row server lanes={lanes}")
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, max_lanes=lanes)
    res = _serve(srv, qs)
    st = srv.stats()
    srv.close()
    _check_per_point(graph, qs, res)
    for r in res:
        assert r["t_submit_ms"] <= r["t_start_ms"] <= r["t_done_ms"]
    assert st["completed"] == len(qs) and st["lanes"] == lanes
    Gd.close()


@pytest.mark.parametrize("streams", [1, 3, 4])
def test_pruned_server_matches_oracle(tpm, graph, streams):
    """Pruned mode with `streams` requests in flight: per-point bytes equal the oracle,
    extracted paths pass the exact checker, and a burst keeps several requests in flight."""
    rng = np.random.default_rng(61 + streams)
    qs = _queries(rng, 30, graph.num_colors, 1, 9, wild=0.1)
    say(f"case pruned server streams={streams}")
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, prune_queries=1, extract_paths=1, streams=streams)
    res = _serve(srv, qs)
    st = srv.stats()
    srv.close()
    _check_per_point(graph, qs, res)
    assert st["completed"] == len(qs) and st["steps"] == len(qs) and st["streams"] == streams
    assert st["prune_ms"] > 0 and st["sieve_ms"] > 0 and st["row_points"] == 0
    assert 1 <= st["inflight_peak"] <= streams
    # queue metrics: the burst waited in the queue; all drained at the end
    assert st["queued_peak"] >= 1 and st["queued"] == 0 and st["inflight"] == 0
    for q, r in zip(qs, res):
        k = len(q["multiset"])
        if r["found"] and k >= 2:
            assert r["path_status"] == tpm.TPM_OK
            assert pyref.check_path(graph, q["multiset"], r["path_vertices"][:k],
                                    r["path_edges"][:k - 1])
    Gd.close()


@pytest.mark.parametrize("prune", [0, 1])
def test_server_alone_vs_mix(tpm, prune):
    """A probe request gives the same per-point bytes alone and submitted in the middle
    of a stream, and both equal the oracle; paths of every hit check out."""
    g = G.uniform_graph(400, 4000, 50, 3, 9)
    Gd = tpm.Graph.from_temporal(g)
    probe = {"multiset": [0, 1, 2, 0], "seed": 4242}
    srv = tpm.Server(Gd, extract_paths=1, prune_queries=prune, streams=3 if prune else 0)
    alone = _serve(srv, [probe])[0]
    rng = np.random.default_rng(3)
    mix = _queries(rng, 25, 3, 2, 8)
    tickets = []
    t_probe = None
    for i, q in enumerate(mix):
        tickets.append(srv.submit(q["multiset"], q["seed"], per_point=True))
        if i == 12:
            t_probe = srv.submit(probe["multiset"], probe["seed"], per_point=True)
    got = {r["ticket"]: r for r in srv.drain(len(mix) + 1)}
    srv.close()
    mixed = got[t_probe]
    assert np.array_equal(mixed["per_point"], alone["per_point"])
    _check_per_point(g, [probe, probe], [alone, mixed])
    _check_per_point(g, mix, [got[t] for t in tickets])
    for r in list(got.values()) + [alone]:
        if r["found"]:
            assert r["path_status"] == tpm.TPM_OK
    if alone["found"]:
        assert pyref.check_path(g, probe["multiset"], alone["path_vertices"][:4], alone["path_edges"][:3])
    Gd.close()


@pytest.mark.parametrize("prune", [0, 1])
def test_server_cancel(tpm, graph, prune):
    """Cancelled requests end with status TPM_ECANCELLED (those still queued at once);
    every other request of the stream is unaffected and equals the oracle; a finished
    ticket can no longer be cancelled."""
    rng = np.random.default_rng(900 + prune)
    qs = _queries(rng, 30, graph.num_colors, 6, 10)
    say(f"case cancel prune={prune}")
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, prune_queries=prune, streams=2 if prune else 0)
    tickets = [srv.submit(q["multiset"], q["seed"], per_point=True) for q in qs]
    cancel = set(tickets[10::3])
    flags = {t: srv.cancel(t) for t in cancel}
    got = {r["ticket"]: r for r in srv.drain(len(qs), timeout_s=300)}
    assert not srv.cancel(tickets[0])  # already out
    st = srv.stats()
    srv.close()
    n_cancelled = 0
    for t, q in zip(tickets, qs):
        r = got[t]
        if r["status"] == tpm.TPM_ECANCELLED:
            assert t in cancel and flags[t]
            assert "per_point" not in r
            n_cancelled += 1
        else:
            assert r["status"] == 0
            _check_per_point(graph, [q], [r])
    assert n_cancelled >= 1 and st["cancelled"] == n_cancelled and st["completed"] == len(qs)
    Gd.close()


@pytest.mark.parametrize("prune", [0, 1])
def test_server_deadline(tpm, graph, prune):
    """A request whose deadline has passed before it could run ends TPM_ECANCELLED; the
    same query without a deadline equals the oracle."""
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, prune_queries=prune)
    q = {"multiset": [0, 1, 2, 3, 4, 0, 1, 2], "seed": 77}
    # a queue of work ahead of the timed request, so that it waits past its deadline
    ahead = [srv.submit([int(c) for c in np.random.default_rng(i).integers(0, 5, 10)], i)
             for i in range(6)]
    t_late = srv.submit(q["multiset"], q["seed"], per_point=True, deadline_ms=0.001)
    t_ok = srv.submit(q["multiset"], q["seed"], per_point=True)
    got = {r["ticket"]: r for r in srv.drain(len(ahead) + 2, timeout_s=300)}
    st = srv.stats()
    srv.close()
    assert got[t_late]["status"] == tpm.TPM_ECANCELLED
    _check_per_point(graph, [q], [got[t_ok]])
    assert st["cancelled"] == 1
    Gd.close()


def test_pruned_server_refuses_what_cannot_fit(tpm, graph):
    """A state budget too small for any request: submission fails with TPM_ENOMEM and
    the server keeps serving nothing else wrongly; malformed requests are refused."""
    Gd = tpm.Graph.from_temporal(graph)
    srv = tpm.Server(Gd, prune_queries=1, state_bytes=4096)
    with pytest.raises(tpm.TpmError) as e:
        srv.submit([0, 1, 2], 5)
    assert e.value.code == tpm.TPM_ENOMEM
    assert srv.stats()["rejected"] == 1
    for bad in ([], [0] * 17, [graph.num_colors], [-2]):
        with pytest.raises(tpm.TpmError) as e:
            srv.submit(bad, 1)
        assert e.value.code == tpm.TPM_EINVAL
    srv.close()
    # a budget that holds one small request at a time still serves every request
    srv = tpm.Server(Gd, prune_queries=1, streams=3, state_bytes=64 << 20)
    rng = np.random.default_rng(5)
    qs = _queries(rng, 12, graph.num_colors, 2, 5)
    res = _serve(srv, qs)
    st = srv.stats()
    srv.close()
    _check_per_point(graph, qs, res)
    assert st["budget_bytes"] == 64 << 20 and st["completed"] == len(qs)
    Gd.close()
