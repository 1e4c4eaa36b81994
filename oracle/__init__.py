"""CPU oracle for the temporal path-motif sieve.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
bench's CPU-baseline leg.  The product package never imports it, and it imports
nothing from the product package.

Two independent layers live here:
  * `liboracle.so` (tpm_oracle.c): the edge-by-edge evaluation of the temporal
    generating polynomial, Eq. (3), at sieve points, with the constrained
    substitution of Eq. (motif); plus an exact colourful-path existence check.
  * `pyref` (pure Python): brute-force walk enumeration, the literal t-by-n
    recursion of Eq. (3), GF(2^8) by polynomial long division, determinants,
    the path checker and the closed-form false-negative rate.  These pin the C
    oracle.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def lib():
    global _lib
    if _lib is None:
        # TPM_ORACLE_SANITIZED=1 loads the AddressSanitizer/UBSan build instead (the
        # process must have libasan preloaded)
        if os.environ.get("TPM_ORACLE_SANITIZED") == "1":
            path = _build.SAN_LIB
            if not os.path.exists(path):
                _build.build_sanitized()
        else:
            path = os.path.join(_HERE, "liboracle.so")
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(
                    os.path.join(_HERE, "tpm_oracle.c")):
                _build.build()
        L = ctypes.CDLL(path)
        L.or_init.restype = None
        L.or_gf_mul_bits.restype = ctypes.c_uint8
        L.or_gf_mul_bits.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
        L.or_gf_mul.restype = ctypes.c_uint8
        L.or_gf_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
        L.or_mul_table.argtypes = [_u8p]
        L.or_mix64.restype = ctypes.c_uint64
        L.or_mix64.argtypes = [ctypes.c_uint64]
        L.or_fp.restype = ctypes.c_uint8
        L.or_fp.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.or_slots.argtypes = [_i32p, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
        L.or_z.argtypes = [ctypes.c_int32, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                           ctypes.c_uint64, _u8p, _u8p]
        L.or_index_build.restype = ctypes.c_void_p
        L.or_index_build.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p]
        L.or_index_free.argtypes = [ctypes.c_void_p]
        L.or_index_set_eid.argtypes = [ctypes.c_void_p, _i32p]
        L.or_eval.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_int32, ctypes.c_uint64, _u32p,
                              ctypes.c_int64, _u8p, _u8p, ctypes.c_int]
        L.or_sieve.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p,
                               ctypes.c_int32, _i32p, ctypes.c_int32, ctypes.c_uint64, _u8p,
                               _u32p, ctypes.c_int64, _u8p, _u8p, ctypes.c_int]
        L.or_sieve_ex.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p,
                                  _i32p, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                  ctypes.c_uint64, _u8p, _u32p, ctypes.c_int64, _u8p, _u8p,
                                  ctypes.c_int]
        L.or_sieve_em.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p,
                                  _i32p, _u8p, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                  ctypes.c_uint64, _u8p, _u32p, ctypes.c_int64, _u8p, _u8p,
                                  ctypes.c_int]
        L.or_static_sieve.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p,
                                      ctypes.c_int32, _i32p, ctypes.c_int32, ctypes.c_uint64,
                                      _u8p, _u8p, ctypes.c_int]
        L.or_sieve_vc.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p, _i32p,
                                  _i32p, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                  ctypes.c_uint64, _u32p, ctypes.c_int64, _u8p, _u8p, ctypes.c_int]
        L.or_colorful_exists.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p, _i32p,
                                         _i32p, ctypes.c_int32, _i32p, ctypes.c_int32]
        L.or_init()
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else ctypes.cast(None, t)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def gf_mul_bits(a: int, b: int) -> int:
    return int(lib().or_gf_mul_bits(a, b))


def mul_table() -> np.ndarray:
    t = np.empty((256, 256), dtype=np.uint8)
    lib().or_mul_table(t.ctypes.data_as(_u8p))
    return t


def mix64(x: int) -> int:
    return int(lib().or_mix64(x & 0xFFFFFFFFFFFFFFFF))


def fp(seed: int, tag: int, a: int, b: int) -> int:
    return int(lib().or_fp(seed & 0xFFFFFFFFFFFFFFFF, tag, a, b))


def slots(M, q: int):
    M = _c32(M)
    off = np.empty(q, dtype=np.int32)
    mu = np.empty(q, dtype=np.int32)
    rc = lib().or_slots(_p(M, _i32p), len(M), q, _p(off, _i32p), _p(mu, _i32p))
    if rc:
        raise ValueError("multiset names a colour outside [0, q)")
    return off, mu


def zvals(g, M, seed: int, mask=None) -> np.ndarray:
    M = _c32(M)
    k = len(M)
    z = np.empty((g.n, k), dtype=np.uint8)
    color = _c32(g.color)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().or_z(g.n, _p(color, _i32p), g.num_colors, _p(M, _i32p), k,
                    seed & 0xFFFFFFFFFFFFFFFF, _p(mk, _u8p), _p(z, _u8p))
    if rc:
        raise ValueError("bad query")
    return z


def sieve(g, M, seed: int, points=None, mask=None, loc: bool = False, nthreads: int = 0,
          transit=None, delay=None, emask=None):
    """P(A) for the given sieve points (default: all 2^k).  Returns the per-point
    array, or (per_point, per_edge_localisation) when loc=True (localisation is
    XOR-ed over the given points).  transit (per edge) and delay (per vertex) select
    the variant with transition and delay times (section "Path motif problem with
    delays"): an edge reaches its head at tau + transit, and a walk leaves a vertex w
    at time tau only if it arrived by tau - delay(w); defaults 0 and 1.  emask (per
    edge, nullable): edges with emask 0 are not in the graph (the others keep their
    index, hence their y)."""
    M = _c32(M)
    k = len(M)
    if points is None:
        points = np.arange(1 << k, dtype=np.uint32)
    points = np.ascontiguousarray(points, dtype=np.uint32)
    out = np.empty(points.shape[0], dtype=np.uint8)
    lc = np.empty(g.m, dtype=np.uint8) if loc else None
    src, dst, tau, color = _c32(g.src), _c32(g.dst), _c32(g.tau), _c32(g.color)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    tr = None if transit is None else _c32(transit)
    dl = None if delay is None else _c32(delay)
    em = None if emask is None else np.ascontiguousarray(emask, dtype=np.uint8)
    if em is not None and em.shape[0] != g.m:
        raise ValueError("emask needs one entry per edge")
    rc = lib().or_sieve_em(g.n, g.m, _p(src, _i32p), _p(dst, _i32p), _p(tau, _i32p),
                           _p(tr, _i32p), _p(dl, _i32p), _p(em, _u8p), _p(color, _i32p), g.num_colors,
                           _p(M, _i32p), k, seed & 0xFFFFFFFFFFFFFFFF, _p(mk, _u8p),
                           _p(points, _u32p), points.shape[0], _p(out, _u8p), _p(lc, _u8p),
                           nthreads)
    if rc:
        raise RuntimeError(f"oracle failed ({rc})")
    return (out, lc) if loc else out


def sd_instance(g, s: int, d: int):
    """(s,d)-COLORFUL-PATH reduction (section "Solving COLORFUL-PATH and
    (s,d)-COLORFUL-PATH"): g with colour q on s and q + 1 on d (q + 2 colours), and the
    edge mask that removes s's in-edges and d's out-edges, so that a matching path of
    the multiset M + {q, q + 1} starts at s and ends at d.  Returns (graph, emask) for
    `sieve(..., emask=emask)`."""
    if not (0 <= s < g.n and 0 <= d < g.n) or s == d:
        raise ValueError("bad (s, d)")
    color = np.array(g.color, dtype=np.int32, copy=True)
    q = int(g.num_colors)
    color[s], color[d] = q, q + 1
    emask = ((np.asarray(g.dst) != s) & (np.asarray(g.src) != d)).astype(np.uint8)
    return dataclasses.replace(g, color=color, num_colors=q + 2), emask


def static_sieve(g, M, seed: int, mask=None, nthreads: int = 0) -> np.ndarray:
    """Static vertex-localised sieve (preprocessing step (ii), Eq. (1)): per vertex u,
    S_u = sum over the 2^k points and the k walk positions l of F_{u,l} G_{u,l} on the
    static instance (one arc per ordered pair with a temporal edge, loops dropped, y
    keyed by the pair's smallest input edge id, tag 4).  Nonzero only at vertices of a
    static path whose colours match M."""
    M = _c32(M)
    S = np.empty(g.n, dtype=np.uint8)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().or_static_sieve(g.n, g.m, _p(_c32(g.src), _i32p), _p(_c32(g.dst), _i32p),
                               _p(_c32(g.color), _i32p), g.num_colors, _p(M, _i32p), len(M),
                               seed & 0xFFFFFFFFFFFFFFFF, _p(mk, _u8p), _p(S, _u8p), nthreads)
    if rc:
        raise RuntimeError(f"oracle failed ({rc})")
    return S


def vc_sieve(g, C, seed: int, points=None, loc: bool = False, nthreads: int = 0, transit=None,
             delay=None):
    """VC-PATH-MOTIF (section "Extending the framework"): C is the ordered tuple of k
    colours; the polynomial keeps x_u at level 1 only for c(u) = C[0] and level l only
    edges (v -> u) with c(v) = C[l-2], c(u) = C[l-1]; the substitution is that of the
    multiset of C.  Returns per-point values (and per-edge localisation)."""
    C = _c32(C)
    k = len(C)
    if points is None:
        points = np.arange(1 << k, dtype=np.uint32)
    points = np.ascontiguousarray(points, dtype=np.uint32)
    out = np.empty(points.shape[0], dtype=np.uint8)
    lc = np.empty(g.m, dtype=np.uint8) if loc else None
    src, dst, tau, color = _c32(g.src), _c32(g.dst), _c32(g.tau), _c32(g.color)
    tr = None if transit is None else _c32(transit)
    dl = None if delay is None else _c32(delay)
    rc = lib().or_sieve_vc(g.n, g.m, _p(src, _i32p), _p(dst, _i32p), _p(tau, _i32p),
                           _p(tr, _i32p), _p(dl, _i32p), _p(color, _i32p), g.num_colors,
                           _p(C, _i32p), k, seed & 0xFFFFFFFFFFFFFFFF, _p(points, _u32p),
                           points.shape[0], _p(out, _u8p), _p(lc, _u8p), nthreads)
    if rc:
        raise RuntimeError(f"oracle failed ({rc})")
    return (out, lc) if loc else out


def sieve_total(g, M, seed: int, mask=None, nthreads: int = 0, transit=None, delay=None) -> int:
    pp = sieve(g, M, seed, mask=mask, nthreads=nthreads, transit=transit, delay=delay)
    return int(np.bitwise_xor.reduce(pp)) if pp.size else 0


def vertex_sieve(g, M, seed: int, mask=None, nthreads: int = 0, transit=None,
                 delay=None) -> np.ndarray:
    """Vertex-localised sieve (section "Vertex-localization"): Q_u = sum over all
    sieve points A of P_{u,k,t}(z^A).  P_{u,k,t} is the sum of the last-level
    contributions of u's in-edges, so Q_u is the XOR of the per-edge localisation
    over the edges that end at u.  k >= 2."""
    if len(M) < 2:
        raise ValueError("vertex localisation needs k >= 2")
    _, lc = sieve(g, M, seed, mask=mask, loc=True, nthreads=nthreads, transit=transit,
                  delay=delay)
    q = np.zeros(g.n, dtype=np.uint8)
    np.bitwise_xor.at(q, np.asarray(g.dst, dtype=np.int64), lc)
    return q


def time_buckets(g, M, seed: int, mask=None, nthreads: int = 0, transit=None, delay=None):
    """Per-timestamp split of the sieve: for each distinct arrival time t (ascending;
    arrival = timestamp without transition times), B(t) = XOR of the per-edge
    localisation over the edges arriving at t.  A walk's last edge arrives last, so
    the XOR of B over times <= t is the sieve restricted to walks that finish by t.
    k >= 2."""
    if len(M) < 2:
        raise ValueError("time buckets need k >= 2")
    _, lc = sieve(g, M, seed, mask=mask, loc=True, nthreads=nthreads, transit=transit,
                  delay=delay)
    arr = np.asarray(g.tau, dtype=np.int64)
    if transit is not None:
        arr = arr + np.asarray(transit, dtype=np.int64)
    times, inv = np.unique(arr, return_inverse=True)
    b = np.zeros(times.shape[0], dtype=np.uint8)
    np.bitwise_xor.at(b, inv, lc)
    return times.astype(np.int32), b


def optimum_time(g, M, seed: int, reps: int = 1, nthreads: int = 0, transit=None,
                 delay=None) -> int:
    """Section "Finding optimum timestamp": the smallest t such that the sieve over
    walks finishing by t is nonzero, minimised over `reps` seeds (seed_r = seed +
    r * 0x9E3779B97F4A7C15, as for decide); -1 if none.  The prefix XOR of the time
    buckets is zero before the first nonzero bucket, so that bucket's time is the
    first t with a nonzero prefix."""
    best = -1
    for r in range(reps):
        sr = (seed + r * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        times, b = time_buckets(g, M, sr, nthreads=nthreads, transit=transit, delay=delay)
        nz = np.nonzero(b)[0]
        if nz.size:
            t = int(times[nz[0]])
            best = t if best < 0 else min(best, t)
    return best


class Index:
    """Reusable oracle index (in-lists sorted by time) for repeated evaluations;
    keeps references to the arrays it borrows.

    keep_colours (optional): index only the edges whose two endpoints have one of these
    colours, the paper's preprocessing step (i).  A vertex whose colour is not in the
    multiset has z = 0 (Eq. (motif)), so every term of a walk through it vanishes and
    such edges change no value; the kept edges keep their input indices as fingerprint
    keys.  eval() then accepts only multisets whose colours are all kept (no
    wildcards)."""

    def __init__(self, g, keep_colours=None):
        self.g = g
        self.keep = None
        src, dst, tau = _c32(g.src), _c32(g.dst), _c32(g.tau)
        self._eid = None
        if keep_colours is not None:
            self.keep = set(int(c) for c in keep_colours)
            incol = np.zeros(max(1, int(g.num_colors)), dtype=bool)
            incol[sorted(self.keep)] = True
            color = np.asarray(g.color)
            sel = np.nonzero(incol[color[src]] & incol[color[dst]])[0]
            self._eid = sel.astype(np.int32)
            src, dst, tau = src[sel], dst[sel], tau[sel]
        self._src, self._dst, self._tau = src, dst, tau
        self.m = int(src.shape[0])
        self._h = lib().or_index_build(g.n, self.m, _p(self._src, _i32p), _p(self._dst, _i32p),
                                       _p(self._tau, _i32p))
        if not self._h:
            raise MemoryError("oracle index")
        if self._eid is not None:
            lib().or_index_set_eid(ctypes.c_void_p(self._h), _p(self._eid, _i32p))

    def eval(self, M, seed: int, points, mask=None, nthreads: int = 0) -> np.ndarray:
        if self.keep is not None and not all(int(c) in self.keep for c in M):
            raise ValueError("the multiset has a colour (or a wildcard) whose edges were dropped")
        z = zvals(self.g, M, seed, mask)
        points = np.ascontiguousarray(points, dtype=np.uint32)
        out = np.empty(points.shape[0], dtype=np.uint8)
        rc = lib().or_eval(ctypes.c_void_p(self._h), _p(z, _u8p), len(M),
                           seed & 0xFFFFFFFFFFFFFFFF, _p(points, _u32p), points.shape[0],
                           _p(out, _u8p), None, nthreads)
        if rc:
            raise RuntimeError(f"oracle failed ({rc})")
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_index_free(ctypes.c_void_p(self._h))
            self._h = None


def colorful_exists(g, M) -> int:
    M = _c32(M)
    src, dst, tau, color = _c32(g.src), _c32(g.dst), _c32(g.tau), _c32(g.color)
    return int(lib().or_colorful_exists(g.n, g.m, _p(src, _i32p), _p(dst, _i32p),
                                        _p(tau, _i32p), _p(color, _i32p), g.num_colors,
                                        _p(M, _i32p), len(M)))
