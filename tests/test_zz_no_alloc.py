"""GPU: tpm_sieve_noalloc (the sieve on the library's fixed per-GPU scratch block, no
allocation) gives exactly tpm_sieve's per-point values and total, on two calls in a row
(the second with a smaller graph and query), refuses a graph whose state cannot fit the
block, and keeps working after the refusal."""

import sys

import numpy as np
import pytest

import oracle
from synth import graphs as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2001_07158_amd import tpm
    return torch, tpm


def _noalloc(torch, Gd, M, seed):
    k = len(M)
    pp = torch.full((1 << k,), 0xAB, dtype=torch.uint8, device="cuda")
    tot = torch.full((1,), 0xCD, dtype=torch.uint8, device="cuda")
    err = torch.full((1,), 0x7777, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    Gd.sieve_noalloc(M, seed, tot, per_point=pp, error_flags=err, stream=st)
    st.synchronize()
    return pp.cpu().numpy(), int(tot.cpu()[0]), int(err.cpu()[0])


def test_noalloc_matches_sieve_two_calls(env):
    torch, tpm = env
    # call 1: a 1e5-edge power-law graph, k = 10 (1024 points)
    g1 = G.chung_lu_graph(20_000, 100_000, 2.5, 500, 8, 3)
    M1 = [0, 1, 1, 2, 3, 4, 5, 6, 7, 7]
    say(f"case noalloc call 1: n={g1.n} m={g1.m} k={len(M1)}")
    G1 = tpm.Graph.from_temporal(g1)
    want_pp, want_tot = G1.sieve(M1, 11)
    pp, tot, err = _noalloc(torch, G1, M1, 11)
    assert err == 0
    assert np.array_equal(pp, want_pp), np.nonzero(pp != want_pp)[0][:8]
    assert tot == want_tot
    G1.close()
    # call 2: a smaller graph and query; the block keeps call 1's contents
    g2 = G.uniform_graph(1_000, 10_000, 100, 4, 5)
    M2 = [0, 0, 1, 2, 3]
    say(f"case noalloc call 2: n={g2.n} m={g2.m} k={len(M2)}")
    G2 = tpm.Graph.from_temporal(g2)
    want_pp, want_tot = G2.sieve(M2, 12)
    pp, tot, err = _noalloc(torch, G2, M2, 12)
    assert err == 0
    assert np.array_equal(pp, want_pp), np.nonzero(pp != want_pp)[0][:8]
    assert tot == want_tot
    assert np.array_equal(pp, oracle.sieve(g2, M2, 12))
    G2.close()


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_noalloc_small_k_and_edgeless(env, k):
    torch, tpm = env
    g = G.uniform_graph(300, 2_000, 30, 3, 40 + k)
    M = [int(c) for c in np.random.default_rng(k).integers(0, 3, k)]
    say(f"case noalloc small k={k}")
    Gd = tpm.Graph.from_temporal(g)
    pp, tot, err = _noalloc(torch, Gd, M, 5)
    want = oracle.sieve(g, M, 5)
    assert err == 0 and np.array_equal(pp, want) and tot == int(np.bitwise_xor.reduce(want))
    assert np.array_equal(pp, Gd.sieve(M, 5)[0])
    Gd.close()
    e = G.TemporalGraph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                        np.zeros(5, np.int32), 1)
    Ge = tpm.Graph.from_temporal(e)
    pp, tot, err = _noalloc(torch, Ge, [0] * k, 5)
    assert np.array_equal(pp, Ge.sieve([0] * k, 5)[0]) and tot == Ge.sieve([0] * k, 5)[1] and err == 0
    Ge.close()


def test_noalloc_refuses_what_cannot_fit(env):
    torch, tpm = env
    # 2e7 vertices: 16 bytes of z per vertex alone exceed the 256 MiB block
    n = 20_000_000
    g = G.TemporalGraph(n, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                        np.array([1, 2], np.int32), np.zeros(n, np.int32), 2)
    say("case noalloc refusal")
    Gd = tpm.Graph.from_temporal(g)
    tot = torch.zeros(1, dtype=torch.uint8, device="cuda")
    with pytest.raises(tpm.TpmError) as e:
        Gd.sieve_noalloc([0, 0, 0], 1, tot)
    assert e.value.code == tpm.TPM_ENOMEM
    with pytest.raises(tpm.TpmError) as e:
        Gd.sieve_noalloc([0, 5], 1, tot)  # colour out of range
    assert e.value.code == tpm.TPM_EINVAL
    Gd.close()
    # still serves a graph that fits
    g2 = G.uniform_graph(200, 1_000, 20, 2, 8)
    G2 = tpm.Graph.from_temporal(g2)
    pp, t2, err = _noalloc(torch, G2, [0, 1, 1], 3)
    assert err == 0 and np.array_equal(pp, oracle.sieve(g2, [0, 1, 1], 3))
    G2.close()
