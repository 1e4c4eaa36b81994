"""CPU: the identities behind level 2's coefficient form (no GPU, no library).

x_u^A = XOR over j in A of z_u[j] is linear in A's indicator, so level 2's running
value of v's in-list (XOR over its positions q of x_{src q}^A * y_q * x_v^A) equals
x_v^A * (XOR over j in A of W[j]) with W[j] = XOR over q of y_q * z_{src q}[j]; the
row expansion evaluates that product per lane as K + linear + pairwise terms; W is a
segmented XOR scan computed in blocks whose carries are scanned apart.  Each is checked
here against the direct definition on random inputs, in GF(2^8) with modulus 0x11D.
"""

import numpy as np


def gmul(a, b):
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        if a & 0x100:
            a ^= 0x11D
        b >>= 1
    return r


def xrow(zrow, A, k):
    x = 0
    for j in range(k):
        if (A >> j) & 1:
            x ^= zrow[j]
    return x


def test_level2_running_value_is_a_product_of_linear_forms():
    rng = np.random.default_rng(11)
    for k in (3, 5, 8):
        n = 7
        z = rng.integers(0, 256, (n, k)).tolist()
        v = 2
        srcs = rng.integers(0, n, 9).tolist()
        ys = rng.integers(0, 256, 9).tolist()
        W = [0] * k
        acc = [0] * (1 << k)
        for s, y in zip(srcs, ys):
            for j in range(k):
                W[j] ^= gmul(y, z[s][j])
            for A in range(1 << k):
                acc[A] ^= gmul(gmul(xrow(z[s], A, k), y), xrow(z[v], A, k))
            for A in range(1 << k):
                assert acc[A] == gmul(xrow(z[v], A, k), xrow(W, A, k))


def test_row_expansion_by_lanes():
    """A row of 2^k points, lane l making points 16 l + b: K + XOR of L_i over b's
    bits + XOR of q_ij over b's pairs equals x^A S^A."""
    rng = np.random.default_rng(12)
    for k in range(4, 11):
        for _ in range(3):
            z = rng.integers(0, 256, k).tolist()
            W = rng.integers(0, 256, k).tolist()
            z[int(rng.integers(0, k))] = 0
            for lane in range(1 << (k - 4)):
                xh = sh = 0
                for h in range(k - 4):
                    if (lane >> h) & 1:
                        xh ^= z[4 + h]
                        sh ^= W[4 + h]
                Lc = [gmul(z[i], sh ^ W[i]) ^ gmul(xh, W[i]) for i in range(4)]
                q = {(a, b): gmul(z[a], W[b]) ^ gmul(z[b], W[a])
                     for a in range(4) for b in range(a + 1, 4)}
                val = [gmul(xh, sh)] + [0] * 15
                for b in range(1, 16):
                    lo = (b & -b).bit_length() - 1
                    rest = b & (b - 1)
                    u = Lc[lo]
                    for j in range(lo + 1, 4):
                        if (rest >> j) & 1:
                            u ^= q[(lo, j)]
                    val[b] = val[rest] ^ u
                for b in range(16):
                    A = 16 * lane + b
                    assert val[b] == gmul(xrow(z, A, k), xrow(W, A, k)), (k, lane, b)


def test_segmented_scan_in_blocks():
    """Blocks of B positions: an in-block segmented scan, then the carry into a block
    from the inclusive scan of block aggregates under (a, b) -> (b.head ? b.v : a.v ^
    b.v, a.head | b.head), applied to the positions before the block's first head."""
    rng = np.random.default_rng(13)
    for trial in range(30):
        m = int(rng.integers(1, 600))
        B = int(rng.choice([4, 16, 64]))
        dst = np.sort(rng.integers(0, int(rng.integers(1, 40)), m))
        vals = rng.integers(0, 2**32, m, dtype=np.uint64)
        want = np.zeros(m, dtype=np.uint64)
        for p in range(m):
            head = p == 0 or dst[p] != dst[p - 1]
            want[p] = vals[p] if head else want[p - 1] ^ vals[p]
        nb = (m + B - 1) // B
        local = np.zeros(m, dtype=np.uint64)
        opened = np.zeros(m, dtype=bool)
        agg = []
        for b in range(nb):
            v, f = 0, False
            for p in range(b * B, min(m, b * B + B)):
                head = p == 0 or dst[p] != dst[p - 1]
                v = vals[p] if head else v ^ vals[p]
                f = f or head
                local[p], opened[p] = v, not f
            agg.append((v, f))
        scanned = []
        for v, f in agg:
            if scanned and not f:
                v = scanned[-1][0] ^ v
            scanned.append((v, f or (bool(scanned) and scanned[-1][1])))
        got = local.copy()
        for p in range(m):
            b = p // B
            if opened[p] and b > 0:
                got[p] ^= scanned[b - 1][0]
        assert np.array_equal(got, want), trial
