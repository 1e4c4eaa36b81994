"""Pure-Python references that pin the C oracle (test infrastructure only).

Everything here is written independently of tpm_oracle.c:
  * GF(2^8) multiplication as a carry-less product of integers followed by
    polynomial long division by x^8+x^4+x^3+x^2+1;
  * the SplitMix64 output mix, written from its published definition;
  * the slot sets and the substitution z_{u,j} of Eq. (motif);
  * brute-force enumeration of temporal walks (the definition of the generating
    polynomial: one monomial per walk, section "Monomial encoding of a temporal
    walk");
  * the literal recursion of Eq. (3) over (vertex, length, time);
  * determinants over GF(2^8) by Gaussian elimination;
  * the exact path checker and the closed-form false-negative probability.
"""

from __future__ import annotations

from functools import lru_cache
from itertools import product

import numpy as np

MASK64 = (1 << 64) - 1
FIELD_POLY = 0x11D  # x^8 + x^4 + x^3 + x^2 + 1


# --------------------------------------------------------------------------- GF(2^8)
def clmul(a: int, b: int) -> int:
    """Carry-less (GF(2)[x]) product of two polynomials given as bit masks."""
    r = 0
    i = 0
    while b >> i:
        if (b >> i) & 1:
            r ^= a << i
        i += 1
    return r


def poly_mod(a: int, m: int = FIELD_POLY) -> int:
    """Remainder of polynomial a modulo m (long division over GF(2))."""
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def gmul(a: int, b: int) -> int:
    return poly_mod(clmul(a, b))


@lru_cache(maxsize=None)
def mul_table() -> np.ndarray:
    t = np.zeros((256, 256), dtype=np.uint8)
    for a in range(256):
        for b in range(256):
            t[a, b] = gmul(a, b)
    return t


def ginv(a: int) -> int:
    if a == 0:
        raise ZeroDivisionError
    r = 1
    for _ in range(254):  # a^254 = a^-1 in a field of 256 elements
        r = gmul(r, a)
    return r


def det(Z) -> int:
    """Determinant over GF(2^8) by Gaussian elimination (characteristic 2: no signs)."""
    M = [list(map(int, row)) for row in Z]
    k = len(M)
    d = 1
    for c in range(k):
        piv = next((r for r in range(c, k) if M[r][c]), None)
        if piv is None:
            return 0
        if piv != c:
            M[c], M[piv] = M[piv], M[c]
        d = gmul(d, M[c][c])
        inv = ginv(M[c][c])
        for r in range(c + 1, k):
            if M[r][c]:
                f = gmul(M[r][c], inv)
                M[r] = [M[r][j] ^ gmul(f, M[c][j]) for j in range(k)]
    return d


# --------------------------------------------------------------------------- fingerprints
def mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood 2014; constants of the
    published generator)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def fp(seed: int, tag: int, a: int, b: int) -> int:
    key = ((tag << 56) ^ (a << 32) ^ b) & MASK64
    return mix64((seed & MASK64) ^ mix64(key)) & 0xFF


TAG_Y, TAG_V, TAG_W, TAG_STATIC = 1, 2, 3, 4


def slots(M, q: int):
    """Distinct colours of M ascending; colour s owns mu(s) consecutive slots.  Entries
    -1 are wildcards: they sort first and own slots 0 .. wc - 1."""
    mu = [0] * q
    for c in M:
        if int(c) >= 0:
            mu[int(c)] += 1
    off = [-1] * q
    nxt = sum(1 for c in M if int(c) == -1)
    for s in range(q):
        if mu[s]:
            off[s] = nxt
            nxt += mu[s]
    return off, mu


def zvals(g, M, seed: int, mask=None) -> np.ndarray:
    k = len(M)
    off, mu = slots(M, g.num_colors)
    w = [[fp(seed, TAG_W, d, j) for j in range(k)] for d in range(k)]
    z = np.zeros((g.n, k), dtype=np.uint8)
    wild = list(range(sum(1 for c in M if int(c) == -1)))  # every vertex owns these too
    for u in range(g.n):
        c = int(g.color[u])
        if mask is not None and not mask[u]:
            continue
        mine = wild + list(range(off[c], off[c] + mu[c]))
        for j in range(k):
            acc = 0
            for d in mine:
                acc ^= gmul(fp(seed, TAG_V, d, u), w[d][j])
            z[u, j] = acc
    return z


def colours_match(colours, M) -> bool:
    """A vertex-colour list matches M when each vertex can take its own colour or a
    wildcard (-1) so that the multiset is M."""
    if len(colours) != len(M):
        return False
    need = {}
    for c in M:
        if int(c) >= 0:
            need[int(c)] = need.get(int(c), 0) + 1
    have = {}
    for c in colours:
        have[int(c)] = have.get(int(c), 0) + 1
    return all(have.get(c, 0) >= n for c, n in need.items())


def subset_values(z: np.ndarray) -> np.ndarray:
    """X[u, A] = sum_{j in A} z[u, j] for every subset A of the k labels."""
    n, k = z.shape
    X = np.zeros((n, 1 << k), dtype=np.uint8)
    for A in range(1 << k):
        for j in range(k):
            if (A >> j) & 1:
                X[:, A] ^= z[:, j]
    return X


# --------------------------------------------------------------------------- walks
def temporal_walks(g, k: int, transit=None, delay=None):
    """All temporal walks with k vertices: lists of edge ids (e_1..e_{k-1}) with
    dst(e_l) = src(e_{l+1}) and tau strictly increasing.  k = 1: one per vertex.
    With transit (per edge) / delay (per vertex): e_{l+1} may follow e_l through w
    iff tau(e_l) + transit(e_l) <= tau(e_{l+1}) - delay(w) (defaults 0 and 1)."""
    if k == 1:
        return [((u,), ()) for u in range(g.n)]
    out_edges = [[] for _ in range(g.n)]
    for e in range(g.m):
        out_edges[int(g.src[e])].append(e)
    res = []

    def extend(edges):
        if len(edges) == k - 1:
            verts = (int(g.src[edges[0]]),) + tuple(int(g.dst[e]) for e in edges)
            res.append((verts, tuple(edges)))
            return
        last = edges[-1]
        w = int(g.dst[last])
        arr = int(g.tau[last]) + (int(transit[last]) if transit is not None else 0)
        dl = int(delay[w]) if delay is not None else 1
        for e in out_edges[w]:
            if arr <= int(g.tau[e]) - dl:
                extend(edges + [e])

    for e in range(g.m):
        extend([e])
    return res


def brute_vc_per_point(g, C, seed: int) -> np.ndarray:
    """VC-PATH-MOTIF by its definition: the sum over temporal walks whose l-th vertex
    has colour C[l-1] of their monomials, at every sieve point (substitution of the
    multiset of C)."""
    k = len(C)
    T = mul_table()
    X = subset_values(zvals(g, C, seed))
    acc = np.zeros(1 << k, dtype=np.uint8)
    for verts, edges in temporal_walks(g, k):
        if any(int(g.color[w]) != int(C[l]) for l, w in enumerate(verts)):
            continue
        v = X[verts[0]].copy()
        for l, e in enumerate(edges, start=1):
            v = T[v, fp(seed, TAG_Y, l, e)]
            v = T[v, X[verts[l]]]
        acc ^= v
    return acc


def has_vc_path(g, C) -> bool:
    for verts, _ in temporal_walks(g, len(C)):
        if len(set(verts)) == len(verts) and all(int(g.color[w]) == int(C[l]) for l, w in enumerate(verts)):
            return True
    return False


def brute_per_point(g, M, seed: int, mask=None, transit=None, delay=None,
                    emask=None) -> np.ndarray:
    """P(A) for every A as the sum over temporal walks of their monomials,
    x_{w_1} y_{e_1,1} x_{w_2} ... y_{e_{k-1},k-1} x_{w_k}, evaluated at z^A.
    emask (per edge): walks through an edge with emask 0 are left out."""
    k = len(M)
    T = mul_table()
    X = subset_values(zvals(g, M, seed, mask))
    acc = np.zeros(1 << k, dtype=np.uint8)
    for verts, edges in temporal_walks(g, k, transit, delay):
        if emask is not None and not all(emask[e] for e in edges):
            continue
        v = X[verts[0]].copy()
        for l, e in enumerate(edges, start=1):
            v = T[v, fp(seed, TAG_Y, l, e)]
            v = T[v, X[verts[l]]]
        acc ^= v
    return acc


def sd_paths(g, s: int, d: int, M):
    """(s,d)-COLORFUL-PATH by its definition: the temporal paths s -> ... -> d with
    len(M) + 2 vertices whose internal vertices' colours are the multiset M."""
    k = len(M) + 2
    res = []
    for verts, edges in temporal_walks(g, k):
        if verts[0] == s and verts[-1] == d and len(set(verts)) == k and \
                colours_match([int(g.color[u]) for u in verts[1:-1]], M):
            res.append((verts, edges))
    return res


def paths_total(g, paths, M, seed: int) -> int:
    """Sum of y(P) det(Z_P) over the given paths (Z from the multiset M on g)."""
    z = zvals(g, M, seed)
    tot = 0
    for verts, edges in paths:
        y = 1
        for l, e in enumerate(edges, start=1):
            y = gmul(y, fp(seed, TAG_Y, l, e))
        tot ^= gmul(y, det([z[u] for u in verts]))
    return tot


def static_arcs(g) -> dict:
    """The static instance: one arc (v, u) per ordered pair joined by a temporal edge,
    v != u, mapped to the smallest input edge id among those edges."""
    arcs = {}
    for e in range(g.m):
        v, u = int(g.src[e]), int(g.dst[e])
        if v != u and (v, u) not in arcs:
            arcs[(v, u)] = e
    return arcs


def static_walks(g, k: int):
    """All walks with k vertices along the static arcs (vertex tuples)."""
    arcs = static_arcs(g)
    out = [[] for _ in range(g.n)]
    for (v, u) in arcs:
        out[v].append(u)
    walks = [(u,) for u in range(g.n)]
    for _ in range(k - 1):
        walks = [w + (u,) for w in walks for u in out[w[-1]]]
    return walks, arcs


def brute_static_vertex(g, M, seed: int):
    """Per vertex u: the sum over static paths P with k = len(M) vertices through u
    of y(P) det(Z_P), y(P) = prod_l fp(seed, 4, l, arc id of the l-th arc)."""
    k = len(M)
    z = zvals(g, M, seed)
    walks, arcs = static_walks(g, k)
    S = np.zeros(g.n, dtype=np.uint8)
    for w in walks:
        if len(set(w)) != k:
            continue
        y = 1
        for l in range(1, k):
            y = gmul(y, fp(seed, TAG_STATIC, l, arcs[(w[l - 1], w[l])]))
        v = gmul(y, det([z[u] for u in w]))
        for u in w:
            S[u] ^= v
    return S


def brute_static_visits(g, M, seed: int):
    """Per vertex u: sum over points A and over static walks W with k vertices of
    (number of visits of W to u) * (the monomial of W at z^A)."""
    k = len(M)
    T = mul_table()
    X = subset_values(zvals(g, M, seed))
    walks, arcs = static_walks(g, k)
    S = np.zeros(g.n, dtype=np.uint8)
    for w in walks:
        v = X[w[0]].copy()
        for l in range(1, k):
            v = T[v, fp(seed, TAG_STATIC, l, arcs[(w[l - 1], w[l])])]
            v = T[v, X[w[l]]]
        tot = int(np.bitwise_xor.reduce(v))
        for u in w:
            S[u] ^= tot
    return S


def brute_paths_total(g, M, seed: int, mask=None) -> int:
    """Q as the sum over temporal *paths* P of y(P) * det(Z_P), Z_P[s][j] = z_{w_s,j}
    (the sieve over A turns the monomial's product into a permanent = determinant
    in characteristic 2, and walks that repeat a vertex cancel)."""
    k = len(M)
    z = zvals(g, M, seed, mask)
    tot = 0
    for verts, edges in temporal_walks(g, k):
        if len(set(verts)) != k:
            continue
        y = 1
        for l, e in enumerate(edges, start=1):
            y = gmul(y, fp(seed, TAG_Y, l, e))
        tot ^= gmul(y, det([z[u] for u in verts]))
    return tot


def brute_paths_by_end(g, M, seed: int, mask=None):
    """Per end vertex u: sum over temporal paths P ending at u of y(P) det(Z_P);
    and per last-edge time t: the same sum over paths whose last edge has time t.
    Returns (per_vertex [n], {t: value})."""
    k = len(M)
    z = zvals(g, M, seed, mask)
    per_v = np.zeros(g.n, dtype=np.uint8)
    per_t = {}
    for verts, edges in temporal_walks(g, k):
        if len(set(verts)) != k:
            continue
        y = 1
        for l, e in enumerate(edges, start=1):
            y = gmul(y, fp(seed, TAG_Y, l, e))
        v = gmul(y, det([z[u] for u in verts]))
        per_v[verts[-1]] ^= v
        t = int(g.tau[edges[-1]])
        per_t[t] = per_t.get(t, 0) ^ v
    return per_v, per_t


def brute_optimum_time(g, M) -> int:
    """Smallest possible largest timestamp over temporal paths matching M (-1 if
    none): exhaustive search."""
    want = sorted(int(c) for c in M)
    best = -1
    for verts, edges in temporal_walks(g, len(M)):
        if len(set(verts)) == len(verts) and sorted(int(g.color[u]) for u in verts) == want:
            t = int(g.tau[edges[-1]])
            best = t if best < 0 else min(best, t)
    return best


def ec_per_point(g, M, seed: int, times) -> np.ndarray:
    """EC-PATH-MOTIF (section "Extending the framework"): the generating polynomial
    whose level l uses only edges at the prescribed time j_{l-1}, evaluated at every
    sieve point: P_1(u) = x_u, P_l(u) = x_u * sum over edges (v -> u) at time j_{l-1}
    of y_{e,l-1} P_{l-1}(v); the value is the sum over u of P_k(u).  times = (j_1 <
    ... < j_{k-1})."""
    k = len(M)
    times = [int(t) for t in times]
    assert len(times) == k - 1 and all(a < b for a, b in zip(times, times[1:]))
    T = mul_table()
    X = subset_values(zvals(g, M, seed))  # [n][2^k]
    out = np.zeros(1 << k, dtype=np.uint8)
    for A in range(1 << k):
        P = X[:, A].copy()
        for l in range(2, k + 1):
            nxt = np.zeros(g.n, dtype=np.uint8)
            for e in range(g.m):
                if int(g.tau[e]) == times[l - 2]:
                    u, v = int(g.dst[e]), int(g.src[e])
                    nxt[u] ^= T[T[X[u, A], fp(seed, TAG_Y, l - 1, e)], P[v]]
            P = nxt
        out[A] = np.bitwise_xor.reduce(P) if g.n else 0
    return out


def literal_eq3_table(g, M, seed: int, mask=None, X=None) -> np.ndarray:
    """Eq. (3) exactly as written, over (length l, vertex u, time i), i = 0..t:
    P[1][u][i] = x_u;  P[l][u][0] = 0 for l >= 2;
    P[l][u][i] = x_u * sum over edges e = (v -> u, i) of y_{e,l-1} P[l-1][v][i-1]
                 + P[l][u][i-1].
    Returns the array P[l, u, i, A] for l = 1..k (index 0 unused), A = all points.
    `X` (optional) overrides the vertex values X[u, A]."""
    k = len(M)
    T = mul_table()
    if X is None:
        X = subset_values(zvals(g, M, seed, mask))
    t = g.tmax
    npts = X.shape[1]
    in_at = {}
    for e in range(g.m):
        in_at.setdefault((int(g.dst[e]), int(g.tau[e])), []).append(e)
    P = np.zeros((k + 1, g.n, t + 1, npts), dtype=np.uint8)
    for u in range(g.n):
        P[1, u, :, :] = X[u]
    for l in range(2, k + 1):
        for i in range(1, t + 1):
            for u in range(g.n):
                s = np.zeros(npts, dtype=np.uint8)
                for e in in_at.get((u, i), []):
                    v = int(g.src[e])
                    s ^= T[fp(seed, TAG_Y, l - 1, e), P[l - 1, v, i - 1]]
                P[l, u, i] = T[X[u], s] ^ P[l, u, i - 1]
    return P


def literal_eq3_per_point(g, M, seed: int, mask=None) -> np.ndarray:
    """P_{k,t}(A) = sum_u P[k][u][t] from the literal recursion."""
    k = len(M)
    P = literal_eq3_table(g, M, seed, mask)
    out = np.zeros(P.shape[-1], dtype=np.uint8)
    for u in range(g.n):
        out ^= P[k, u, g.tmax if g.m else 0]
    return out


def has_matching_path(g, M, transit=None, delay=None) -> bool:
    for verts, _ in temporal_walks(g, len(M), transit, delay):
        if len(set(verts)) == len(verts) and colours_match([g.color[u] for u in verts], M):
            return True
    return False


def check_path(g, M, verts, edges, transit=None, delay=None) -> bool:
    """Exact check of an extracted witness: k distinct vertices, k-1 edges whose
    endpoints match consecutive vertices, strictly increasing timestamps (or, with
    transition / delay times, each edge leaving after the previous one arrived plus
    the vertex's delay), and vertex colours equal to the multiset M."""
    k = len(M)
    verts = [int(v) for v in verts]
    edges = [int(e) for e in edges]
    if len(verts) != k or len(edges) != k - 1 or len(set(verts)) != k:
        return False
    for v in verts:
        if v < 0 or v >= g.n:
            return False
    for l, e in enumerate(edges):
        if e < 0 or e >= g.m:
            return False
        if int(g.src[e]) != verts[l] or int(g.dst[e]) != verts[l + 1]:
            return False
        if l:
            prev = edges[l - 1]
            arr = int(g.tau[prev]) + (int(transit[prev]) if transit is not None else 0)
            dl = int(delay[verts[l]]) if delay is not None else 1
            if not arr <= int(g.tau[e]) - dl:
                return False
    return colours_match([g.color[v] for v in verts], M)


def unique_witness_detect_prob(M) -> float:
    """P(Q != 0) when exactly one temporal path matches M: Q = y(P) det(V) det(W)
    with y(P) a product of k-1 independent uniform bytes, W a uniform k x k
    matrix, V block-diagonal with one uniform mu(s) x mu(s) block per colour."""
    k = len(M)
    p = (255 / 256) ** (k - 1)
    for i in range(1, k + 1):
        p *= 1 - 256.0 ** (-i)
    counts = {}
    for c in M:
        counts[int(c)] = counts.get(int(c), 0) + 1
    for mu in counts.values():
        for i in range(1, mu + 1):
            p *= 1 - 256.0 ** (-i)
    return p


def all_subsets(k: int):
    return list(product([0, 1], repeat=k))
