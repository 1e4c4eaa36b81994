"""Pins for the oracle's GF(2^8) arithmetic and fingerprint hash (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import pyref


@pytest.fixture(scope="module")
def T():
    return oracle.mul_table().astype(np.int64)


def test_bitserial_matches_long_division_on_all_pairs():
    # C shift-and-add multiply vs Python carry-less product + polynomial long division
    assert np.array_equal(oracle.mul_table(), pyref.mul_table())
    for a, b in [(0, 0), (1, 0x53), (0x53, 0xCA), (0xFF, 0xFF)]:
        assert oracle.gf_mul_bits(a, b) == pyref.gmul(a, b)


def test_reduction_polynomial_0x11d():
    # x^7 * x = x^8 = x^4 + x^3 + x^2 + 1
    assert oracle.gf_mul_bits(0x80, 0x02) == 0x1D
    assert pyref.poly_mod(0x100) == 0x1D


def test_field_axioms_pairs(T):
    a = np.arange(256)
    assert np.array_equal(T, T.T)  # commutative
    assert np.array_equal(T[1], a)  # identity
    assert not T[0].any()  # zero annihilates
    # every nonzero element has exactly one inverse
    for x in range(1, 256):
        assert np.count_nonzero(T[x] == 1) == 1
    # no zero divisors
    assert np.count_nonzero(T[1:, 1:] == 0) == 0


def test_field_axioms_all_triples(T):
    a = np.arange(256)
    # associativity: (a*b)*c == a*(b*c) for all 2^24 triples
    ab = T[a[:, None], a[None, :]]  # [a, b]
    lhs = T[ab[:, :, None], a[None, None, :]]
    rhs = T[a[:, None, None], T[a[:, None], a[None, :]][None, :, :]]
    assert np.array_equal(lhs, rhs)
    # distributivity: a*(b^c) == a*b ^ a*c
    bc = a[:, None] ^ a[None, :]
    lhs = T[a[:, None, None], bc[None, :, :]]
    rhs = T[a[:, None], a[None, :]][:, :, None] ^ T[a[:, None], a[None, :]][:, None, :]
    assert np.array_equal(lhs, rhs)


def test_generator_and_inverse(T):
    # 0x02 generates the multiplicative group (order 255)
    seen, x = set(), 1
    for _ in range(255):
        x = int(T[x, 2])
        seen.add(x)
    assert x == 1 and len(seen) == 255
    # a * a^254 = 1
    for a in range(1, 256):
        p = 1
        for _ in range(254):
            p = int(T[p, a])
        assert int(T[a, p]) == 1


def test_splitmix64_published_output():
    # SplitMix64 with state 0: first output = mix(0 + golden gamma)
    assert oracle.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert pyref.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert oracle.mix64(0) == 0


def test_hash_c_matches_python():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        z = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        assert oracle.mix64(z) == pyref.mix64(z)
    for _ in range(2000):
        seed = int(rng.integers(0, 2**63))
        tag = int(rng.integers(1, 4))
        a = int(rng.integers(0, 16))
        b = int(rng.integers(0, 2**32))
        assert oracle.fp(seed, tag, a, b) == pyref.fp(seed, tag, a, b)


def test_fingerprint_low_byte_uniform():
    # chi-square over 256 bins for y fingerprints of consecutive edges
    seed = 12345
    vals = np.array([pyref.fp(seed, 1, 3, e) for e in range(65536)])
    counts = np.bincount(vals, minlength=256)
    chi2 = float(((counts - 256.0) ** 2 / 256.0).sum())
    # 255 degrees of freedom: mean 255, sd ~22.6; 6 sd band
    assert 120 < chi2 < 400
