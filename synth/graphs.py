"""Temporal graph generators (seeded, numpy only).

A temporal graph here is a directed edge list (src[e], dst[e], tau[e]) with
tau >= 1, plus one colour per vertex, as in the paper's terminology section
(temporal edges are triples (u, v, j) with j a positive integer timestamp) and
its path-motif problem statement (vertex-coloured temporal graph).  Edge e is
identified by its index in these arrays.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class TemporalGraph:
    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    tau: np.ndarray  # int32 [m], >= 1
    color: np.ndarray  # int32 [n]
    num_colors: int

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def tmax(self) -> int:
        return int(self.tau.max()) if self.m else 0

    def copy(self) -> "TemporalGraph":
        return TemporalGraph(self.n, self.src.copy(), self.dst.copy(), self.tau.copy(),
                             self.color.copy(), self.num_colors)


def _redraw_self_loops(rng, src, dst, draw_src, draw_dst):
    bad = np.nonzero(src == dst)[0]
    while bad.size:
        src[bad] = draw_src(bad.size)
        dst[bad] = draw_dst(bad.size)
        bad = bad[src[bad] == dst[bad]]
    return src, dst


def uniform_graph(n: int, m: int, t: int, q: int, seed: int,
                  self_loops: bool = False) -> TemporalGraph:
    """Endpoints uniform over [0, n), no self-loops unless asked, tau ~ U[1, t],
    colours ~ U[0, q)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m, dtype=np.int64)
    dst = rng.integers(0, n, m, dtype=np.int64)
    if not self_loops and n > 1:
        src, dst = _redraw_self_loops(rng, src, dst,
                                      lambda s: rng.integers(0, n, s),
                                      lambda s: rng.integers(0, n, s))
    tau = rng.integers(1, t + 1, m, dtype=np.int64)
    color = rng.integers(0, q, n, dtype=np.int64)
    return TemporalGraph(n, src.astype(np.int32), dst.astype(np.int32),
                         tau.astype(np.int32), color.astype(np.int32), q)


def regular_graph(n: int, d: int, t: int, q: int, seed: int) -> TemporalGraph:
    """Random d-regular undirected multigraph by the configuration model (n d stubs,
    a uniform random pairing; n d must be even), one timestamp per edge ~ U[1, t],
    colours ~ U[0, q).  The edge list holds each undirected edge once (u, v); build
    the device graph with the undirected flag.  The pairing may leave a few loops
    and parallel edges, as the model does."""
    if (n * d) % 2:
        raise ValueError("n d must be even")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    src, dst = stubs[0::2], stubs[1::2]
    m = src.shape[0]
    tau = rng.integers(1, t + 1, m, dtype=np.int64)
    color = rng.integers(0, q, n, dtype=np.int64)
    return TemporalGraph(n, src.astype(np.int32), dst.astype(np.int32), tau.astype(np.int32),
                         color.astype(np.int32), q)


def _alias_sampler(rng, weights: np.ndarray):
    """Draws indices with probability proportional to `weights` (Walker's alias
    method, Vose's construction)."""
    n = weights.shape[0]
    prob = weights.astype(np.float64) * (n / weights.sum())
    accept = np.ones(n, dtype=np.float64)
    alias = np.arange(n, dtype=np.int64)
    small = list(np.nonzero(prob < 1.0)[0])
    large = list(np.nonzero(prob >= 1.0)[0])
    p = prob.tolist()
    while small and large:
        s = small.pop()
        l = large.pop()
        accept[s] = p[s]
        alias[s] = l
        p[l] -= 1.0 - p[s]
        (small if p[l] < 1.0 else large).append(l)

    def draw(size: int) -> np.ndarray:
        out = np.empty(size, dtype=np.int64)
        step = 1 << 24
        for lo in range(0, size, step):
            hi = min(size, lo + step)
            i = rng.integers(0, n, hi - lo)
            u = rng.random(hi - lo)
            out[lo:hi] = np.where(u < accept[i], i, alias[i])
        return out

    return draw


def chung_lu_graph(n: int, m: int, beta: float, t: int, q: int, seed: int) -> TemporalGraph:
    """Directed Chung-Lu graph with power-law expected out- and in-degrees.

    Vertex weights w_i = (i+1)^(-1/(beta-1)); the out-weights and the in-weights
    are two independent random permutations of them.  Each edge draws its source
    with probability proportional to the out-weight and its destination with
    probability proportional to the in-weight (alias tables); a self-loop is redrawn.  Timestamps
    are uniform on [1, t] and colours uniform on [0, q)."""
    rng = np.random.default_rng(seed)
    base = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (beta - 1.0))
    w_out = base[rng.permutation(n)]
    w_in = base[rng.permutation(n)]
    draw_src = _alias_sampler(rng, w_out)
    draw_dst = _alias_sampler(rng, w_in)
    src = draw_src(m)
    dst = draw_dst(m)
    src, dst = _redraw_self_loops(rng, src, dst, draw_src, draw_dst)
    tau = rng.integers(1, t + 1, m, dtype=np.int64)
    color = rng.integers(0, q, n, dtype=np.int64)
    return TemporalGraph(n, src.astype(np.int32), dst.astype(np.int32),
                         tau.astype(np.int32), color.astype(np.int32), q)


def paper_toy_graph() -> TemporalGraph:
    """The three-vertex worked example of the temporal generating polynomial
    (section 'Generating polynomial for temporal walks' and its figure): undirected
    edges {v1,v2} and {v2,v3}, each present at times 1 and 2.  Undirected edges are
    given as two arcs.  Vertices v1, v2, v3 are 0, 1, 2; one colour (0) for all."""
    arcs = []
    for (a, b) in [(0, 1), (1, 2)]:
        for j in (1, 2):
            arcs.append((a, b, j))
            arcs.append((b, a, j))
    src = np.array([a for a, _, _ in arcs], dtype=np.int32)
    dst = np.array([b for _, b, _ in arcs], dtype=np.int32)
    tau = np.array([j for _, _, j in arcs], dtype=np.int32)
    return TemporalGraph(3, src, dst, tau, np.zeros(3, dtype=np.int32), 1)


def random_tiny_graph(rng: np.random.Generator, n_max: int = 12, m_max: int = 40,
                      t_max: int = 6, q_max: int = 4, allow_self_loops: bool = True) -> TemporalGraph:
    """A small random temporal multigraph for brute-force comparisons: duplicate
    arcs, self-loops and equal timestamps are all allowed on purpose."""
    n = int(rng.integers(1, n_max + 1))
    m = int(rng.integers(0, m_max + 1))
    t = int(rng.integers(1, t_max + 1))
    q = int(rng.integers(1, q_max + 1))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if not allow_self_loops and n > 1:
        src, dst = _redraw_self_loops(rng, src.astype(np.int64), dst.astype(np.int64),
                                      lambda s: rng.integers(0, n, s), lambda s: rng.integers(0, n, s))
        src = src.astype(np.int32)
        dst = dst.astype(np.int32)
    tau = rng.integers(1, t + 1, m).astype(np.int32)
    color = rng.integers(0, q, n).astype(np.int32)
    return TemporalGraph(n, src, dst, tau, color, q)


def relabel_timestamps(g: TemporalGraph, rng: np.random.Generator) -> TemporalGraph:
    """Apply a random strictly increasing map to the timestamps (keeps their order,
    the paper compresses timestamps the same way when it loads data)."""
    h = g.copy()
    if g.m == 0:
        return h
    vals = np.unique(g.tau)
    gaps = rng.integers(1, 50, vals.size)
    newvals = np.cumsum(gaps)
    lut = dict(zip(vals.tolist(), newvals.tolist()))
    h.tau = np.array([lut[int(x)] for x in g.tau], dtype=np.int32)
    return h


def append_isolated(g: TemporalGraph, extra: int, rng: np.random.Generator) -> TemporalGraph:
    h = g.copy()
    h.n = g.n + extra
    h.color = np.concatenate([g.color, rng.integers(0, g.num_colors, extra).astype(np.int32)])
    return h


def static_to_temporal_layers(n: int, edges: list[tuple[int, int]], k: int) -> TemporalGraph:
    """The construction in the NP-hardness proof for temporal k-path: every static
    edge is copied at each timestamp 1..k-1 (here as two arcs per undirected edge).
    A static path with k vertices exists iff a temporal one does."""
    s, d, tt = [], [], []
    for (a, b) in edges:
        for j in range(1, k):
            s += [a, b]
            d += [b, a]
            tt += [j, j]
    return TemporalGraph(n, np.array(s, dtype=np.int32), np.array(d, dtype=np.int32),
                         np.array(tt, dtype=np.int32), np.zeros(n, dtype=np.int32), 1)
