"""GPU parity: the HIP sieve through the C ABI against the CPU oracle, bit for bit.

All sieve values are exact GF(2^8) elements, so the bar is equality of every
per-point byte (and of the per-edge localisation where it is requested)."""

import os
import sys

import numpy as np
import pytest

import oracle
from oracle import pyref
from synth import graphs as G
from synth import make_config_graph, make_config_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_2001_07158_amd import tpm as _tpm
    return _tpm


def _check(tpm, g, M, seed, mask=None, chunk=0, tile_edges=0, label=""):
    say(f"case {label}: n={g.n} m={g.m} k={len(M)} seed={seed} chunk={chunk} "
        f"T={tile_edges} mask={'y' if mask is not None else 'n'}")
    Gd = tpm.Graph.from_temporal(g, tile_edges=tile_edges)
    pp, tot = Gd.sieve(M, seed, mask=mask, chunk=chunk)
    want = oracle.sieve(g, M, seed, mask=mask)
    assert np.array_equal(pp, want), f"{label}: per-point mismatch at {np.nonzero(pp != want)[0][:8]}"
    assert tot == int(np.bitwise_xor.reduce(want))
    Gd.close()
    return tot


def test_tiny_config_all_points(tpm):
    g = make_config_graph("tiny")
    M = make_config_query("tiny")
    nz = 0
    for seed in (1, 2, 3, 20010715):
        nz += _check(tpm, g, M, seed, label="tiny") != 0
    assert nz >= 2  # ~7.8e3 expected matches: the total is nonzero for most seeds


def test_paper_toy_graph(tpm):
    g = G.paper_toy_graph()
    for seed in range(1, 6):
        _check(tpm, g, [0, 0, 0], seed, label="toy k=3")
        Gd = tpm.Graph.from_temporal(g)
        assert Gd.sieve([0, 0, 0, 0], seed)[1] == 0  # no 4-vertex temporal path
        Gd.close()


def test_random_small_graphs(tpm):
    rng = np.random.default_rng(99)
    for it in range(120):
        g = G.random_tiny_graph(rng, n_max=40, m_max=200, t_max=8, q_max=4)
        k = int(rng.integers(1, 8))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        mask = None if it % 4 else (rng.random(g.n) < 0.8).astype(np.uint8)
        _check(tpm, g, M, int(rng.integers(0, 2**63)), mask=mask, label=f"rand{it}")


def test_empty_and_degenerate(tpm):
    rng = np.random.default_rng(5)
    # no edges
    g = G.TemporalGraph(4, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                        np.array([0, 1, 0, 1], np.int32), 2)
    for k in (1, 2, 3):
        _check(tpm, g, [0] * k, 7, label=f"empty k={k}")
    # one vertex, self-loops only
    g = G.TemporalGraph(1, np.zeros(5, np.int32), np.zeros(5, np.int32),
                        np.arange(1, 6, dtype=np.int32), np.zeros(1, np.int32), 1)
    for k in (1, 2, 3):
        _check(tpm, g, [0] * k, 3, label=f"selfloops k={k}")
    # all edges at one timestamp: no walk longer than one edge
    g = G.uniform_graph(50, 400, 1, 2, 17)
    _check(tpm, g, [0, 1], 4, label="one-time k=2")
    assert _check(tpm, g, [0, 1, 0], 4, label="one-time k=3") == 0
    # every vertex masked
    g = G.uniform_graph(30, 200, 5, 2, 18)
    _check(tpm, g, [0, 1, 1], 5, mask=np.zeros(30, np.uint8), label="all-masked")
    del rng


@pytest.mark.parametrize("T", [1, 2, 7, 16, 64, 256, 1000, 4096])
def test_tile_shapes_with_hubs(tpm, T):
    # power-law in-degrees: long in-lists split over many tiles (look-back path)
    g = G.chung_lu_graph(3000, 60000, 2.5, 50, 3, 1234)
    M = [0, 1, 2, 0, 1, 2]
    _check(tpm, g, M, 42, tile_edges=T, label=f"hubs T={T}")


@pytest.mark.parametrize("chunk", [128, 256, 512])
@pytest.mark.parametrize("T", [1, 5, 64])
def test_slot_tiles_with_hubs(tpm, chunk, T):
    """Rows of 128..512 points run several tiles per wave, one per slot: hub in-lists
    split over many tiny tiles put a piece's predecessor in the same wave (look-back
    within a ticket), tile counts leave idle slots, and tiles of one ticket differ in
    length."""
    g = G.chung_lu_graph(3000, 60000, 2.5, 50, 3, 1234)
    M = [0, 1, 2, 0, 1, 2, 0, 1, 2]  # k = 9, 512 points
    _check(tpm, g, M, 43, chunk=chunk, tile_edges=T, label=f"slot hubs chunk={chunk} T={T}")


@pytest.mark.parametrize("k", [7, 8, 9])
def test_slot_tiles_localisation(tpm, k):
    """Per-edge localisation of the last level at 128-, 256- and 512-point rows, where
    a batch's bytes are reduced across the slot's lanes together."""
    rng = np.random.default_rng(40 + k)
    g = G.chung_lu_graph(1500, 30000, 2.5, 40, 3, 300 + k)
    M = [int(c) for c in rng.integers(0, 3, k)]
    T = int(rng.integers(1, 40))
    say(f"case slot loc k={k} T={T} M={M}")
    Gd = tpm.Graph.from_temporal(g, tile_edges=T)
    pp, tot, loc = Gd.sieve(M, 17 + k, loc=True)
    wpp, wloc = oracle.sieve(g, M, 17 + k, loc=True)
    assert np.array_equal(pp, wpp)
    assert np.array_equal(loc, wloc)
    Gd.close()


@pytest.mark.parametrize("chunk", [4, 16, 64, 256, 512, 1024])
def test_chunk_sizes(tpm, chunk):
    g = G.chung_lu_graph(2000, 30000, 2.5, 40, 4, 77)
    M = [0, 1, 2, 3, 0, 1, 2, 3, 0, 1]  # k = 10, 1024 points
    _check(tpm, g, M, 9, chunk=chunk, label=f"chunk={chunk}")


def test_more_than_one_chunk_k12(tpm):
    g = G.chung_lu_graph(500, 6000, 2.5, 30, 3, 5)
    M = [0, 1, 2] * 4
    _check(tpm, g, M, 11, label="k=12")
    _check(tpm, g, M, 11, chunk=256, label="k=12 chunk 256")


def test_localisation_matches_oracle(tpm):
    rng = np.random.default_rng(3)
    for it in range(10):
        g = G.chung_lu_graph(400, 5000, 2.5, 30, 3, 100 + it)
        M = [int(c) for c in rng.integers(0, 3, int(rng.integers(2, 7)))]
        say(f"case loc{it}: k={len(M)}")
        Gd = tpm.Graph.from_temporal(g, tile_edges=int(rng.integers(1, 300)))
        pp, tot, loc = Gd.sieve(M, 5 + it, loc=True)
        wpp, wloc = oracle.sieve(g, M, 5 + it, loc=True)
        assert np.array_equal(pp, wpp)
        assert np.array_equal(loc, wloc)
        Gd.close()


def test_decide_and_extract_tiny(tpm):
    g = make_config_graph("tiny")
    M = make_config_query("tiny")
    Gd = tpm.Graph.from_temporal(g)
    assert Gd.decide(M, 1, reps=4)
    for seed in (1, 2, 3):
        say(f"case extract tiny seed={seed}")
        rc, verts, edges = Gd.extract(M, seed)
        assert rc == tpm.TPM_OK
        assert pyref.check_path(g, M, verts, edges)
    Gd.close()


def test_extract_random_graphs_agree_with_brute_force(tpm):
    rng = np.random.default_rng(8)
    seen_yes = seen_no = 0
    for it in range(60):
        g = G.random_tiny_graph(rng, n_max=12, m_max=40, t_max=6, q_max=3)
        k = int(rng.integers(2, 5))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        exists = pyref.has_matching_path(g, M)
        say(f"case extract rand{it} exists={exists}")
        Gd = tpm.Graph.from_temporal(g)
        rc, verts, edges = Gd.extract(M, 1000 + it, max_reps=12)
        if exists:
            seen_yes += 1
            assert rc == tpm.TPM_OK, it
            assert pyref.check_path(g, M, verts, edges)
        else:
            seen_no += 1
            assert rc == tpm.TPM_NOTFOUND
            assert not Gd.decide(M, it, reps=5)
        Gd.close()
    assert seen_yes > 5 and seen_no > 5


def test_batch_matches_alone(tpm):
    g = G.chung_lu_graph(3000, 40000, 2.5, 60, 6, 9)
    rng = np.random.default_rng(4)
    qs = [{"multiset": [int(c) for c in rng.integers(0, 6, int(rng.integers(3, 9)))],
           "seed": int(rng.integers(0, 2**40))} for _ in range(12)]
    Gd = tpm.Graph.from_temporal(g)
    res = Gd.batch(qs)
    for q, r in zip(qs, res):
        pp, tot = Gd.sieve(q["multiset"], q["seed"])
        assert r["total"] == tot
        assert r["found"] == (tot != 0)
    Gd.close()


def test_k5_config_full(tpm):
    g = make_config_graph("k5")
    M = make_config_query("k5")
    say(f"case k5 full: M={list(M)}")
    _check(tpm, g, M, 20010715, label="k5 full")


def test_graph_stats(tpm):
    g = G.chung_lu_graph(2000, 20000, 2.5, 50, 3, 3)
    Gd = tpm.Graph.from_temporal(g)
    st = Gd.stats()
    # rows = positions some later edge reads (independent count on the host)
    order = np.lexsort((np.arange(g.m), g.tau, g.dst))
    key = g.dst[order].astype(np.int64) * (g.tmax + 2) + g.tau[order]
    q = g.src.astype(np.int64) * (g.tmax + 2) + g.tau
    idx = np.searchsorted(key, q, "left") - 1
    ok = idx >= 0
    ok[ok] &= (key[idx[ok]] // (g.tmax + 2)) == g.src[ok]
    assert st["rows"] == np.unique(idx[ok]).size
    assert st["m"] == g.m and st["n"] == g.n
    assert st["max_in_degree"] == np.bincount(g.dst, minlength=g.n).max()
    Gd.close()


def test_retile_is_bit_identical(tpm):
    g = G.chung_lu_graph(3000, 60000, 2.5, 50, 3, 77)
    M = [0, 1, 2, 0, 1, 2, 0]
    want = oracle.sieve(g, M, 13)
    Gd = tpm.Graph.from_temporal(g)
    for T in (1, 3, 64, 1024, 4096, 200):
        say(f"case retile T={T}")
        Gd.retile(T)
        st = Gd.stats()
        Gf = tpm.Graph.from_temporal(g, tile_edges=T)
        assert st["tiles"] == Gf.stats()["tiles"] and st["slots"] == Gf.stats()["slots"]
        Gf.close()
        pp, tot = Gd.sieve(M, 13)
        assert np.array_equal(pp, want), T
    with pytest.raises(tpm.TpmError):
        Gd.retile(0)
    assert np.array_equal(Gd.sieve(M, 13)[0], want)  # the failed retile kept the tiles
    Gd.close()


@pytest.mark.parametrize("k", [5, 9])
def test_autotune_applies_a_candidate_and_keeps_results(tpm, k):
    g = G.chung_lu_graph(20000, 400000, 2.5, 200, 4, 31)
    M = [int(c) for c in np.random.default_rng(k).integers(0, 4, k)]
    Gd = tpm.Graph.from_temporal(g, tile_edges=7)
    say(f"case autotune k={k}")
    rep = Gd.autotune(k, seed=5)
    cands = rep["candidates"]
    chunks = [min(2**k, 256)] if 2**k < 256 else [c for c in (256, 512, 1024) if c <= 2**k]
    assert len(cands) == 4 * len(chunks)
    assert {(c["tile_edges"], c["chunk"]) for c in cands} == {
        (t, c) for t in (256, 512, 1024, 2048) for c in chunks}
    best = max(cands, key=lambda c: c["rate"])
    assert (rep["tile_edges"], rep["chunk"]) == (best["tile_edges"], best["chunk"])
    Gf = tpm.Graph.from_temporal(g, tile_edges=rep["tile_edges"])
    assert Gd.stats()["tiles"] == Gf.stats()["tiles"]
    Gf.close()
    pp, _ = Gd.sieve(M, 3, chunk=rep["chunk"])
    assert np.array_equal(pp, oracle.sieve(g, M, 3))
    # the same key (architecture, k, log2 m, log2 n) is served from the cache
    Gd.retile(7)
    again = Gd.autotune(k, seed=6)
    assert again["cached"] and not again["candidates"]
    assert (again["tile_edges"], again["chunk"]) == (rep["tile_edges"], rep["chunk"])
    assert np.array_equal(Gd.sieve(M, 3, chunk=again["chunk"])[0], pp)
    Gd.close()


def test_autotune_cache_file(tmp_path):
    """TPM_AUTOTUNE_CACHE keeps results across processes: a second process reads the
    first one's entry and times nothing."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    code = ("import sys; sys.path.insert(0, %r); from synth import graphs as G; "
            "from paper_2001_07158_amd import tpm; "
            "g = G.chung_lu_graph(3000, 30000, 2.5, 50, 4, 8); "
            "Gd = tpm.Graph.from_temporal(g); r = Gd.autotune(6, seed=2); "
            "print(int(r['cached']), r['tile_edges'], r['chunk']); Gd.close()"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    env = dict(os.environ, TPM_AUTOTUNE_CACHE=str(cache))
    say("case autotune cache file")
    out1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out1.returncode == 0, out1.stderr[-2000:]
    c1, t1, ch1 = out1.stdout.split()[-3:]
    assert c1 == "0" and len(cache.read_text().splitlines()) == 1
    out2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out2.returncode == 0, out2.stderr[-2000:]
    assert out2.stdout.split()[-3:] == ["1", t1, ch1]


@pytest.mark.timeout(600)
def test_k10_full_size_sampled_points(tpm):
    """The k = 10 workload at full size (n = 1e6, m = 1e8), in the launch
    configuration the bench times (one 1024-point chunk), against the oracle on 64
    sieve points computed one by one."""
    import os
    g = make_config_graph("k10")
    M = make_config_query("k10")
    seed = 20010715
    say(f"case k10 full: n={g.n} m={g.m} M={list(M)}")
    Gd = tpm.Graph.from_temporal(g)
    pp, tot = Gd.sieve(M, seed)
    assert tot == int(np.bitwise_xor.reduce(pp))
    st = Gd.stats()
    Gd.close()
    # one point per lane (lane L holds points 16 L .. 16 L + 15 of the 1024-point row),
    # at byte position L mod 16 of the lane: every lane and every byte position of a
    # lane's 16 points is checked
    pts = np.array([16 * L + (L % 16) for L in range(64)])
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    say(f"oracle on {pts.size} points, {nthreads} threads (rows={st['rows']})")
    idx = oracle.Index(g)
    want = idx.eval(M, seed, pts.astype(np.uint32), nthreads=nthreads)
    assert np.array_equal(pp[pts], want), (pts, pp[pts], want)


def test_selfreduce_extraction_against_brute_force(tpm):
    """The paper's self-reducibility extraction (group testing + temporal DFS) finds
    a valid path exactly when one exists, also on layered (VC) and delayed graphs."""
    rng = np.random.default_rng(151)
    yes = no = 0
    for it in range(40):
        g = G.random_tiny_graph(rng, n_max=12, m_max=40, t_max=6, q_max=3)
        k = int(rng.integers(2, 5))
        M = [int(c) for c in rng.integers(-1 if it % 5 == 4 else 0, g.num_colors, k)]
        exists = pyref.has_matching_path(g, M)
        Gd = tpm.Graph.from_temporal(g)
        rc, verts, edges, ns = Gd.extract_ex(M, 200 + it, max_reps=6, method=1)
        if exists:
            yes += 1
            assert rc == tpm.TPM_OK, it
            assert pyref.check_path(g, M, verts, edges)
        else:
            no += 1
            assert rc == tpm.TPM_NOTFOUND
        rc2, _, _, ns2 = Gd.extract_ex(M, 200 + it, max_reps=6, method=0)
        assert rc2 == rc
        Gd.close()
    assert yes > 5 and no > 5
    g = G.random_tiny_graph(np.random.default_rng(7), n_max=12, m_max=40, t_max=6, q_max=3)
    tr = np.ones(g.m, np.int32)
    dl = np.zeros(g.n, np.int32)
    for M in ([0, 1], [0, 1, 2], [1, 1, 0]):
        Gd = tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, transit=tr, delay=dl)
        rc, verts, edges, _ = Gd.extract_ex(M, 5, max_reps=6, method=1)
        assert (rc == tpm.TPM_OK) == pyref.has_matching_path(g, M, tr, dl)
        if rc == tpm.TPM_OK:
            assert pyref.check_path(g, M, verts, edges, tr, dl)
        Gd.close()


def test_device_pointer_input(tpm):
    """Graph creation from device arrays (TPM_DEVICE_PTRS) gives the same index and
    results as from host arrays; bad device input is rejected on the device."""
    import torch
    g = G.chung_lu_graph(2000, 30000, 2.5, 40, 4, 161)
    dev = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
           for a in (g.src, g.dst, g.tau, g.color)]
    torch.cuda.synchronize()
    h = tpm.tpm_graph_create(g.n, *[(t.data_ptr(), t.numel()) for t in dev], g.num_colors,
                             flags=tpm.TPM_DEVICE_PTRS)
    M = [0, 1, 2, 3, 0, 1]
    pp, tot = tpm.tpm_sieve(h, M, 5)
    assert np.array_equal(pp, oracle.sieve(g, M, 5))
    host = tpm.Graph.from_temporal(g)
    a, b = tpm.tpm_graph_stats_get(h), host.stats()
    for key in ("rows", "tiles", "slots", "gathers", "segments", "max_in_degree", "tmax"):
        assert a[key] == b[key], key
    host.close()
    tpm.tpm_graph_destroy(h)
    bad = dev[2].clone()
    bad[7] = 0  # timestamp < 1
    with pytest.raises(tpm.TpmError) as ei:
        tpm.tpm_graph_create(g.n, (dev[0].data_ptr(), g.m), (dev[1].data_ptr(), g.m),
                             (bad.data_ptr(), g.m), (dev[3].data_ptr(), g.n), g.num_colors,
                             flags=tpm.TPM_DEVICE_PTRS)
    assert ei.value.code == tpm.TPM_EINVAL


def test_concurrent_sieves_on_streams(tpm):
    """Sieves on one graph from several host threads, each on its own stream (the
    graph is immutable; each call leases its own workspace)."""
    import threading
    import torch
    g = G.chung_lu_graph(3000, 50000, 2.5, 50, 4, 162)
    Gd = tpm.Graph.from_temporal(g)
    qs = [([0, 1, 2, 3, 0, 1, 2][: 3 + i % 5], 10 + i) for i in range(12)]
    want = [oracle.sieve(g, M, s) for M, s in qs]
    got = [None] * len(qs)
    errs = []

    def work(j):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            for i in range(j, len(qs), 3):
                M, s = qs[i]
                got[i] = Gd.sieve(M, s, stream=st)[0]
        except Exception as e:  # reported below
            errs.append(e)

    th = [threading.Thread(target=work, args=(j,)) for j in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for i in range(len(qs)):
        assert np.array_equal(got[i], want[i]), i
    Gd.close()


def test_k16_all_points_tiny(tpm):
    """The largest query size: 65536 sieve points in 64 chunks of 1024."""
    g = G.uniform_graph(60, 500, 30, 4, 163)
    M = [int(c) for c in np.random.default_rng(1).integers(0, 4, 16)]
    _check(tpm, g, M, 77, label="k=16")


def test_vertexloc_extraction_against_brute_force(tpm):
    """The paper's vertex-localisation extraction (Q_u, then reverse temporal DFS from
    a certified end vertex) finds a valid path exactly when one exists, also with
    wildcards, transition / delay times and on layered (VC) graphs."""
    rng = np.random.default_rng(191)
    yes = no = 0
    for it in range(50):
        g = G.random_tiny_graph(rng, n_max=14, m_max=50, t_max=6, q_max=3)
        k = int(rng.integers(2, 6))
        M = [int(c) for c in rng.integers(-1 if it % 5 == 4 else 0, g.num_colors, k)]
        exists = pyref.has_matching_path(g, M)
        say(f"case vertexloc {it}: n={g.n} m={g.m} M={M} exists={exists}")
        Gd = tpm.Graph.from_temporal(g, tile_edges=int(rng.integers(1, 32)))
        rc, verts, edges, ns = Gd.extract_ex(M, 400 + it, max_reps=8, method=2)
        if exists:
            yes += 1
            assert rc == tpm.TPM_OK, it
            assert pyref.check_path(g, M, verts, edges)
            assert 1 <= ns <= 8
        else:
            no += 1
            assert rc == tpm.TPM_NOTFOUND
        Gd.close()
    assert yes > 10 and no > 5
    g = G.random_tiny_graph(np.random.default_rng(7), n_max=12, m_max=40, t_max=6, q_max=3)
    assert g.num_colors == 3
    tr = np.ones(g.m, np.int32)
    dl = np.zeros(g.n, np.int32)
    for M in ([0, 1], [0, 1, 2], [1, 1, 0]):
        Gd = tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, transit=tr, delay=dl)
        rc, verts, edges, _ = Gd.extract_ex(M, 5, max_reps=8, method=2)
        assert (rc == tpm.TPM_OK) == pyref.has_matching_path(g, M, tr, dl)
        if rc == tpm.TPM_OK:
            assert pyref.check_path(g, M, verts, edges, tr, dl)
        Gd.close()


def test_vertexloc_extraction_planted(tpm):
    """A planted 8-vertex path on a Chung-Lu graph: extracted by the reverse DFS from
    one localised sieve; the three methods agree on existence."""
    g = G.chung_lu_graph(3000, 40000, 2.5, 80, 12, 192)
    rng = np.random.default_rng(3)
    k = 8
    verts = [int(v) for v in rng.choice(g.n, k, replace=False)]
    color = g.color.copy()
    M = [int(c) for c in rng.integers(0, 12, k)]
    for v, c in zip(verts, M):
        color[v] = c
    src = np.concatenate([g.src, np.array(verts[:-1], dtype=np.int32)])
    dst = np.concatenate([g.dst, np.array(verts[1:], dtype=np.int32)])
    tau = np.concatenate([g.tau, np.arange(1, k, dtype=np.int32) * 9])
    h = G.TemporalGraph(g.n, src, dst, tau, color, 12)
    Gd = tpm.Graph.from_temporal(h)
    rc, pv, pe, ns = Gd.extract_ex(M, 11, max_reps=8, method=2)
    assert rc == tpm.TPM_OK
    assert pyref.check_path(h, M, pv, pe)
    rc0, pv0, pe0, _ = Gd.extract_ex(M, 11, max_reps=8, method=0)
    assert rc0 == tpm.TPM_OK and pyref.check_path(h, M, pv0, pe0)
    Gd.close()


def test_undirected_graphs(tpm):
    """TPM_UNDIRECTED: each edge also runs dst -> src (input id e + m); results equal the
    oracle's on the explicitly doubled edge list, with and without transition times."""
    rng = np.random.default_rng(195)
    for it in range(30):
        g = G.random_tiny_graph(rng, n_max=30, m_max=150, t_max=8, q_max=4)
        k = int(rng.integers(1, 7))
        M = [int(c) for c in rng.integers(0, g.num_colors, k)]
        tr = rng.integers(0, 3, g.m).astype(np.int32) if it % 3 == 2 else None
        d = G.TemporalGraph(g.n, np.concatenate([g.src, g.dst]), np.concatenate([g.dst, g.src]),
                            np.concatenate([g.tau, g.tau]), g.color, g.num_colors)
        tr2 = None if tr is None else np.concatenate([tr, tr])
        say(f"case undirected {it}: n={g.n} m={g.m} M={M} transit={tr is not None}")
        Gd = tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, transit=tr,
                       undirected=True, tile_edges=int(rng.integers(1, 64)))
        assert Gd.stats()["m"] == 2 * g.m and Gd.stats()["edge_ids"] == 2 * g.m
        pp, tot, loc = Gd.sieve(M, 900 + it, loc=True)
        wpp, wloc = oracle.sieve(d, M, 900 + it, loc=True, transit=tr2)
        assert np.array_equal(pp, wpp), it
        assert np.array_equal(loc, wloc), it
        if k >= 2 and tot:
            rc, verts, edges = Gd.extract(M, 900 + it)
            assert rc == tpm.TPM_OK
            assert pyref.check_path(d, M, verts, edges, tr2)
        Gd.close()


def test_default_tile_size(tpm):
    """Default tiles: min(1024, max(128, m / 4096)); subgraphs choose again for their own
    m; an explicit size or a retile is kept."""
    want = lambda m: min(1024, max(128, m // 4096))  # noqa: E731
    g = G.uniform_graph(5000, 2_000_000, 100, 8, 196)
    Gd = tpm.Graph.from_temporal(g)
    assert Gd.stats()["tile_edges"] == want(g.m)
    Gp = Gd.prune([0, 1])
    assert Gp.stats()["tile_edges"] == want(Gp.stats()["m"])
    Gp.close()
    Gd.retile(300)
    assert Gd.stats()["tile_edges"] == 300
    Gq = Gd.prune([0, 1])
    assert Gq.stats()["tile_edges"] == 300
    Gq.close()
    Gd.close()
    Ge = tpm.Graph.from_temporal(g, tile_edges=777)
    assert Ge.stats()["tile_edges"] == 777
    Ge.close()
