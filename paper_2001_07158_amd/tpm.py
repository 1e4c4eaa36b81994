"""ctypes binding of libtpm.so (include/tpm.h), argument marshalling only.

Every computation runs in the HIP library; if the library is missing this module
raises at import time -- there is no CPU fallback.  Functions keep the C names;
`Graph` and `Server` are thin owners of the handles.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TPM_LIBRARY: path of another build of the library (the host-sanitizer build of the tests)
LIB_PATH = os.environ.get("TPM_LIBRARY") or os.path.join(_HERE, "libtpm.so")

TPM_OK = 0
TPM_NOTFOUND = 1
TPM_PENDING = 2
TPM_EINVAL = -1
TPM_ENOMEM = -2
TPM_EDEVICE = -3
TPM_ECANCELLED = -4
TPM_ECLOSED = -5
TPM_DEVICE_PTRS = 0x1
TPM_UNDIRECTED = 0x2
TPM_WILDCARD = -1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(paper_2001_07158_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class tpm_graph_options(ctypes.Structure):
    _fields_ = [("tile_edges", ctypes.c_int32), ("tile_held", ctypes.c_int32),
                ("transit", ctypes.POINTER(ctypes.c_int32)), ("delay", ctypes.POINTER(ctypes.c_int32))]


class tpm_graph_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("num_colors", ctypes.c_int32),
                ("tmax", ctypes.c_int32), ("rows", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("slots", ctypes.c_int64), ("max_in_degree", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("gathers", ctypes.c_int64),
                ("segments", ctypes.c_int64), ("times", ctypes.c_int64),
                ("edge_ids", ctypes.c_int64), ("tile_edges", ctypes.c_int32)]


class tpm_kernel_time(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("level", ctypes.c_int32),
                ("chunk_points", ctypes.c_int32), ("pad", ctypes.c_int32), ("ms", ctypes.c_double)]


class tpm_tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("streams", ctypes.c_int32)]


class tpm_autotune_report(ctypes.Structure):
    _fields_ = [("tile_edges", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("ncand", ctypes.c_int32), ("cand_tile", ctypes.c_int32 * 12),
                ("cand_chunk", ctypes.c_int32 * 12), ("cand_rate", ctypes.c_double * 12),
                ("cached", ctypes.c_int32)]


class tpm_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("row_points", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("prune_ms", ctypes.c_double), ("sieve_ms", ctypes.c_double),
                ("extract_ms", ctypes.c_double), ("cancelled", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("inflight_peak", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("held_bytes_peak", ctypes.c_int64), ("trims", ctypes.c_int64),
                ("gpu_wait_ms", ctypes.c_double), ("queued", ctypes.c_int32),
                ("queued_peak", ctypes.c_int32), ("inflight", ctypes.c_int32), ("pad", ctypes.c_int32)]


class tpm_query(ctypes.Structure):
    _fields_ = [("multiset", _i32p), ("k", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("want_path", ctypes.c_int32), ("per_point", _u8p), ("deadline_ms", ctypes.c_double)]


class tpm_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("found", ctypes.c_int32), ("total", ctypes.c_uint8),
                ("path_status", ctypes.c_int32), ("path_vertices", ctypes.c_int32 * 16),
                ("path_edges", ctypes.c_int64 * 15), ("ticket", ctypes.c_uint64),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double)]


class tpm_server_config(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_int64), ("max_lanes", ctypes.c_int32),
                ("extract_paths", ctypes.c_int32), ("prune_queries", ctypes.c_int32),
                ("streams", ctypes.c_int32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_vp = ctypes.c_void_p
_sig("tpm_graph_create", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp,
                                         ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(_vp)])
_sig("tpm_graph_create_ex", ctypes.c_int32,
     [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_uint32,
      ctypes.POINTER(tpm_graph_options), ctypes.POINTER(_vp)])
_sig("tpm_graph_destroy", None, [_vp])
_sig("tpm_graph_stats_get", ctypes.c_int32, [_vp, ctypes.POINTER(tpm_graph_stats)])
_sig("tpm_graph_retile", ctypes.c_int32, [_vp, ctypes.c_int32])
_sig("tpm_graph_layer", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.POINTER(_vp)])
_sig("tpm_graph_vertex_ids", ctypes.c_int32, [_vp, _i32p])
_sig("tpm_graph_sd", ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_vp)])
_sig("tpm_extract_optimum", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i64p])
_sig("tpm_static_sieve", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _u8p])
_sig("tpm_graph_prune_static", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64,
                                               ctypes.c_int32, ctypes.POINTER(_vp)])
_sig("tpm_graph_prune", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.POINTER(_vp)])
_sig("tpm_graph_prune_ex", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                           ctypes.POINTER(_vp)])
_sig("tpm_sieve_vertex", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _u8p, _u8p])
_sig("tpm_time_buckets", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _i32p, _u8p])
_sig("tpm_optimum_time", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.c_int32, _i32p])
_sig("tpm_autotune", ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.POINTER(tpm_autotune_report)])
_sig("tpm_sieve", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _u8p, _u8p, _u8p,
                                  _vp])
_sig("tpm_sieve_ex", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _u8p,
                                     ctypes.POINTER(tpm_tuning), _u8p, _u8p, _u8p, _vp])
_sig("tpm_sieve_noalloc", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, _vp, _vp,
                                              _vp, _vp])
_sig("tpm_decide", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                   _i32p])
_sig("tpm_extract", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                    _i32p, _i64p])
_sig("tpm_extract_ex", ctypes.c_int32, [_vp, _i32p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_int32, _i32p, _i64p, _i64p])
_sig("tpm_batch_run", ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(tpm_query),
                                      ctypes.POINTER(tpm_result), ctypes.POINTER(tpm_tuning)])
_sig("tpm_rainbow_decide", ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                           _i32p, _i32p])
_sig("tpm_server_create", ctypes.c_int32, [_vp, ctypes.POINTER(tpm_server_config),
                                          ctypes.POINTER(_vp)])
_sig("tpm_server_submit", ctypes.c_int32, [_vp, ctypes.POINTER(tpm_query), _u64p])
_sig("tpm_server_poll", ctypes.c_int32, [_vp, ctypes.POINTER(tpm_result), ctypes.c_int32, _i32p])
_sig("tpm_server_cancel", ctypes.c_int32, [_vp, ctypes.c_uint64])
_sig("tpm_server_destroy", None, [_vp])
_sig("tpm_server_stats_get", ctypes.c_int32, [_vp, ctypes.POINTER(tpm_server_stats)])
_sig("tpm_profile_enable", ctypes.c_int32, [ctypes.c_int32])
_sig("tpm_profile_read", ctypes.c_int32, [ctypes.POINTER(tpm_kernel_time), ctypes.c_int32, _i32p])
_sig("tpm_stream_read", ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp])
_sig("tpm_last_error", ctypes.c_char_p, [])
_sig("tpm_version", ctypes.c_char_p, [])

EXPORTED = ["tpm_graph_create", "tpm_graph_create_ex", "tpm_graph_destroy", "tpm_graph_stats_get",
            "tpm_graph_retile", "tpm_autotune", "tpm_graph_prune", "tpm_graph_prune_ex",
            "tpm_graph_layer", "tpm_graph_sd", "tpm_graph_vertex_ids", "tpm_sieve_vertex", "tpm_time_buckets",
            "tpm_optimum_time", "tpm_static_sieve", "tpm_graph_prune_static",
            "tpm_sieve", "tpm_sieve_ex", "tpm_sieve_noalloc", "tpm_decide", "tpm_extract", "tpm_extract_ex",
            "tpm_extract_optimum",
            "tpm_batch_run",
            "tpm_server_create", "tpm_server_submit", "tpm_server_poll", "tpm_server_cancel",
            "tpm_server_destroy",
            "tpm_server_stats_get", "tpm_rainbow_decide",
            "tpm_profile_enable", "tpm_profile_read", "tpm_stream_read", "tpm_last_error",
            "tpm_version"]


class TpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tpm error {code}: {msg}")
        self.code = code


def tpm_last_error() -> str:
    return (_lib.tpm_last_error() or b"").decode()


def tpm_version() -> str:
    return _lib.tpm_version().decode()


def _check(rc: int, ok=(TPM_OK,)) -> int:
    if rc not in ok:
        raise TpmError(rc, tpm_last_error())
    return rc


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, t=_vp):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(t) if t is not _vp else ctypes.c_void_p(a.ctypes.data)
    return a


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(int(stream.cuda_stream))  # torch.cuda.Stream


# ------------------------------------------------------------------ C-named wrappers
def tpm_graph_create(n, src, dst, tau, color, num_colors, flags=0, tile_edges=0, tile_held=0,
                     transit=None, delay=None):
    """Host numpy arrays, or raw device pointers (ints) with flags=TPM_DEVICE_PTRS.
    transit (per edge) and delay (per vertex) are host arrays (nullable)."""
    h = ctypes.c_void_p()
    if flags & TPM_DEVICE_PTRS:
        m = int(src[1])
        ptrs = [ctypes.c_void_p(int(x[0])) for x in (src, dst, tau, color)]
    else:
        src, dst, tau, color = _i32(src), _i32(dst), _i32(tau), _i32(color)
        m = int(src.shape[0])
        if not (dst.shape[0] == m and tau.shape[0] == m and color.shape[0] == n):
            raise ValueError("array lengths do not match n/m")
        ptrs = [_ptr(x) for x in (src, dst, tau, color)]
    tr = None if transit is None else _i32(transit)
    dl = None if delay is None else _i32(delay)
    if tr is not None and tr.shape[0] != m:
        raise ValueError("transit needs one entry per edge")
    if dl is not None and dl.shape[0] != n:
        raise ValueError("delay needs one entry per vertex")
    opt = tpm_graph_options(int(tile_edges), int(tile_held), _ptr(tr, _i32p), _ptr(dl, _i32p))
    _check(_lib.tpm_graph_create_ex(int(n), m, *ptrs, int(num_colors), int(flags),
                                    ctypes.byref(opt), ctypes.byref(h)))
    return h


def tpm_graph_destroy(h) -> None:
    _lib.tpm_graph_destroy(h)


def tpm_graph_stats_get(h) -> dict:
    st = tpm_graph_stats()
    _check(_lib.tpm_graph_stats_get(h, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in tpm_graph_stats._fields_}


def _mask(h, mask):
    """The vertex mask as n bytes (the library reads exactly n of them)."""
    if mask is None:
        return None
    mk = np.ascontiguousarray(mask, dtype=np.uint8)
    n = tpm_graph_stats_get(h)["n"]
    if mk.ndim != 1 or mk.shape[0] != n:
        raise ValueError(f"vertex mask needs {n} entries, got {mk.shape}")
    return mk


def tpm_sieve(h, multiset, seed, mask=None, chunk=0, loc_m=None, stream=None, prune=False):
    """Returns (per_point uint8[2^k], total int) or, with loc_m = number of edges,
    (per_point, total, loc uint8[m])."""
    M = _i32(multiset)
    k = int(M.shape[0])
    pp = np.zeros(1 << k, dtype=np.uint8)
    tot = np.zeros(1, dtype=np.uint8)
    mk = _mask(h, mask)
    loc = None if loc_m is None else np.zeros(max(1, int(loc_m)), dtype=np.uint8)
    tune = tpm_tuning(int(chunk), 0, 1 if prune else 0, 0)
    _check(_lib.tpm_sieve_ex(h, M.ctypes.data_as(_i32p), k, int(seed) & (2**64 - 1),
                             _ptr(mk, _u8p), ctypes.byref(tune), pp.ctypes.data_as(_u8p),
                             tot.ctypes.data_as(_u8p), _ptr(loc, _u8p), _stream_handle(stream)))
    if loc is not None:
        return pp, int(tot[0]), loc[: int(loc_m)]
    return pp, int(tot[0])


def _dev_ptr(x):
    """A device address: an int, or a tensor's data_ptr(); None stays NULL."""
    if x is None:
        return None
    return ctypes.c_void_p(int(x) if isinstance(x, int) else int(x.data_ptr()))


def tpm_sieve_noalloc(h, multiset, seed, total, per_point=None, error_flags=None, stream=None):
    """Enqueues the sieve on `stream` with no allocation; total (1 byte), per_point
    (2^k bytes) and error_flags (4 bytes) are device buffers (tensors or addresses)."""
    M = _i32(multiset)
    _check(_lib.tpm_sieve_noalloc(h, M.ctypes.data_as(_i32p), int(M.shape[0]), int(seed) & (2**64 - 1),
                                  _dev_ptr(per_point), _dev_ptr(total), _dev_ptr(error_flags),
                                  _stream_handle(stream)))


def tpm_stream_read(src, nbytes, out, stream=None) -> None:
    """Streaming read of nbytes of device memory (src, out: tensors or addresses)."""
    _check(_lib.tpm_stream_read(_dev_ptr(src), int(nbytes), _dev_ptr(out), _stream_handle(stream)))


def tpm_decide(h, multiset, seed, reps=1) -> bool:
    M = _i32(multiset)
    found = ctypes.c_int32(0)
    _check(_lib.tpm_decide(h, M.ctypes.data_as(_i32p), int(M.shape[0]), int(seed) & (2**64 - 1),
                           int(reps), ctypes.byref(found)))
    return bool(found.value)


def tpm_extract(h, multiset, seed, max_reps=8):
    """Returns (status, vertices[k], edges[k-1]); status TPM_OK or TPM_NOTFOUND."""
    M = _i32(multiset)
    k = int(M.shape[0])
    pv = np.full(k, -1, dtype=np.int32)
    pe = np.full(max(1, k - 1), -1, dtype=np.int64)
    rc = _check(_lib.tpm_extract(h, M.ctypes.data_as(_i32p), k, int(seed) & (2**64 - 1),
                                 int(max_reps), pv.ctypes.data_as(_i32p), pe.ctypes.data_as(_i64p)),
                ok=(TPM_OK, TPM_NOTFOUND))
    return rc, pv, pe[: k - 1]


def tpm_extract_optimum(h, multiset, seed, reps=4, method=0):
    """Returns (status, t, vertices[k], edges[k-1]): the optimum finishing time and a
    path that finishes by it."""
    M = _i32(multiset)
    k = int(M.shape[0])
    t = ctypes.c_int32(-1)
    pv = np.full(k, -1, dtype=np.int32)
    pe = np.full(max(1, k - 1), -1, dtype=np.int64)
    rc = _check(_lib.tpm_extract_optimum(h, M.ctypes.data_as(_i32p), k, int(seed) & (2**64 - 1),
                                         int(reps), int(method), ctypes.byref(t),
                                         pv.ctypes.data_as(_i32p), pe.ctypes.data_as(_i64p)),
                ok=(TPM_OK, TPM_NOTFOUND))
    return rc, int(t.value), pv, pe[: k - 1]


def tpm_extract_ex(h, multiset, seed, max_reps=8, method=0):
    """Returns (status, vertices[k], edges[k-1], sieves run); method 0 = localisation,
    1 = self-reducibility with temporal DFS."""
    M = _i32(multiset)
    k = int(M.shape[0])
    pv = np.full(k, -1, dtype=np.int32)
    pe = np.full(max(1, k - 1), -1, dtype=np.int64)
    ns = ctypes.c_int64(0)
    rc = _check(_lib.tpm_extract_ex(h, M.ctypes.data_as(_i32p), k, int(seed) & (2**64 - 1),
                                    int(max_reps), int(method), pv.ctypes.data_as(_i32p),
                                    pe.ctypes.data_as(_i64p), ctypes.byref(ns)),
                ok=(TPM_OK, TPM_NOTFOUND))
    return rc, pv, pe[: k - 1], int(ns.value)


def _make_queries(queries, per_point=False):
    """ctypes query array; with per_point, one uint8[2^k] output buffer per query
    (returned in `pps`, kept alive by the caller until the results are out)."""
    keep, pps = [], []
    arr = (tpm_query * len(queries))()
    for i, q in enumerate(queries):
        M = _i32(q["multiset"])
        keep.append(M)
        arr[i].multiset = M.ctypes.data_as(_i32p)
        arr[i].k = int(M.shape[0])
        arr[i].seed = int(q.get("seed", 0)) & (2**64 - 1)
        arr[i].want_path = int(q.get("want_path", 0))
        arr[i].deadline_ms = float(q.get("deadline_ms", 0.0))
        pp = None
        if per_point:
            pp = np.zeros(1 << int(M.shape[0]), dtype=np.uint8)
            arr[i].per_point = pp.ctypes.data_as(_u8p)
        pps.append(pp)
    return arr, keep, pps


def _result_dict(r: tpm_result, per_point=None) -> dict:
    d = {"status": int(r.status), "found": bool(r.found), "total": int(r.total),
         "path_status": int(r.path_status),
         "path_vertices": list(r.path_vertices), "path_edges": list(r.path_edges),
         "ticket": int(r.ticket), "t_submit_ms": r.t_submit_ms, "t_start_ms": r.t_start_ms,
         "t_done_ms": r.t_done_ms}
    if per_point is not None:
        d["per_point"] = per_point
    return d


def tpm_sieve_vertex(h, multiset, seed, mask=None):
    st = tpm_graph_stats_get(h)
    M = _i32(multiset)
    q = np.empty(st["n"], dtype=np.uint8)
    mk = _mask(h, mask)
    _check(_lib.tpm_sieve_vertex(h, _ptr(M, _i32p), len(M), int(seed) & (2**64 - 1),
                                 _ptr(mk, _u8p), _ptr(q, _u8p)))
    return q


def tpm_time_buckets(h, multiset, seed):
    st = tpm_graph_stats_get(h)
    M = _i32(multiset)
    times = np.empty(st["times"], dtype=np.int32)
    b = np.empty(st["times"], dtype=np.uint8)
    _check(_lib.tpm_time_buckets(h, _ptr(M, _i32p), len(M), int(seed) & (2**64 - 1),
                                 _ptr(times, _i32p), _ptr(b, _u8p)))
    return times, b


def tpm_optimum_time(h, multiset, seed, reps=1) -> int:
    M = _i32(multiset)
    t = ctypes.c_int32(0)
    _check(_lib.tpm_optimum_time(h, _ptr(M, _i32p), len(M), int(seed) & (2**64 - 1),
                                 int(reps), ctypes.byref(t)))
    return int(t.value)


def tpm_graph_prune(h, colors=None, times=None):
    """Subgraph on the edges whose endpoints both have a colour in `colors` (None: all)
    and whose timestamp is in `times` (None: all)."""
    c = None if colors is None else _i32(sorted(set(int(x) for x in colors)))
    t = None if times is None else _i32(sorted(set(int(x) for x in times)))
    out = ctypes.c_void_p()
    _check(_lib.tpm_graph_prune_ex(h, _ptr(c, _i32p), 0 if c is None else len(c),
                                   _ptr(t, _i32p), 0 if t is None else len(t), ctypes.byref(out)))
    return out


def tpm_graph_layer(h, tup):
    t = _i32(list(tup))
    out = ctypes.c_void_p()
    _check(_lib.tpm_graph_layer(h, _ptr(t, _i32p), len(t), ctypes.byref(out)))
    return out


def tpm_graph_sd(h, s, d):
    out = ctypes.c_void_p()
    _check(_lib.tpm_graph_sd(h, int(s), int(d), ctypes.byref(out)))
    return out


def tpm_static_sieve(h, multiset, seed):
    """Per-vertex static vertex-localised sieve values (uint8[n])."""
    M = _i32(multiset)
    n = tpm_graph_stats_get(h)["n"]
    out = np.zeros(n, dtype=np.uint8)
    _check(_lib.tpm_static_sieve(h, _ptr(M, _i32p), len(M), int(seed) & (2**64 - 1),
                                 _ptr(out, _u8p)))
    return out


def tpm_graph_prune_static(h, multiset, seed, reps=1):
    M = _i32(multiset)
    out = ctypes.c_void_p()
    _check(_lib.tpm_graph_prune_static(h, _ptr(M, _i32p), len(M), int(seed) & (2**64 - 1),
                                       int(reps), ctypes.byref(out)))
    return out


def tpm_graph_vertex_ids(h):
    n = tpm_graph_stats_get(h)["n"]
    ids = np.empty(n, dtype=np.int32)
    _check(_lib.tpm_graph_vertex_ids(h, _ptr(ids, _i32p)))
    return ids


def tpm_graph_retile(h, tile_edges) -> None:
    _check(_lib.tpm_graph_retile(h, int(tile_edges)))


def tpm_autotune(h, k, seed=1) -> dict:
    rep = tpm_autotune_report()
    _check(_lib.tpm_autotune(h, int(k), int(seed) & (2**64 - 1), ctypes.byref(rep)))
    return {"tile_edges": rep.tile_edges, "chunk": rep.chunk, "cached": bool(rep.cached),
            "candidates": [{"tile_edges": rep.cand_tile[i], "chunk": rep.cand_chunk[i],
                            "rate": rep.cand_rate[i]} for i in range(rep.ncand)]}


def tpm_batch_run(h, queries, chunk=0, use_graph=False, prune=False, streams=0, per_point=False):
    """Results as dicts; with per_point, each carries its query's uint8[2^k] values."""
    arr, _keep, pps = _make_queries(queries, per_point)
    out = (tpm_result * len(queries))()
    tune = tpm_tuning(int(chunk), 1 if use_graph else 0, 1 if prune else 0, int(streams))
    _check(_lib.tpm_batch_run(h, len(queries), arr, out, ctypes.byref(tune)))
    return [_result_dict(out[i], pps[i]) for i in range(len(queries))]


def tpm_rainbow_decide(h, k, seed=1, reps=1):
    """(found, colours) for a temporal path with k distinct colours."""
    found = ctypes.c_int32(0)
    cols = np.zeros(max(1, int(k)), dtype=np.int32)
    _check(_lib.tpm_rainbow_decide(h, int(k), int(seed) & (2**64 - 1), int(reps),
                                   ctypes.byref(found), _ptr(cols, _i32p)))
    return bool(found.value), [int(c) for c in cols[: int(k)]] if found.value else None


def tpm_server_create(h, state_bytes=0, max_lanes=0, extract_paths=0, prune_queries=0, streams=0):
    cfg = tpm_server_config(int(state_bytes), int(max_lanes), int(extract_paths),
                            int(prune_queries), int(streams))
    s = ctypes.c_void_p()
    _check(_lib.tpm_server_create(h, ctypes.byref(cfg), ctypes.byref(s)))
    return s


def tpm_server_submit(s, multiset, seed, want_path=0, per_point=None, deadline_ms=0.0) -> int:
    """per_point: None, or a uint8[2^k] numpy array that the server fills before the
    result is polled (the caller keeps it alive until then)."""
    arr, keep, _ = _make_queries([{"multiset": multiset, "seed": seed, "want_path": want_path,
                                   "deadline_ms": deadline_ms}])
    if per_point is not None:
        if (not isinstance(per_point, np.ndarray) or per_point.dtype != np.uint8
                or not per_point.flags["C_CONTIGUOUS"] or per_point.size != (1 << int(arr[0].k))):
            raise ValueError("per_point must be a contiguous uint8 array of 2^k entries")
        arr[0].per_point = per_point.ctypes.data_as(_u8p)
    t = ctypes.c_uint64(0)
    _check(_lib.tpm_server_submit(s, ctypes.byref(arr[0]), ctypes.byref(t)))
    del keep
    return int(t.value)


def tpm_server_poll(s, max_results=64):
    out = (tpm_result * max_results)()
    n = ctypes.c_int32(0)
    _check(_lib.tpm_server_poll(s, out, int(max_results), ctypes.byref(n)), ok=(TPM_OK, TPM_PENDING))
    return [_result_dict(out[i]) for i in range(n.value)]


def tpm_server_cancel(s, ticket) -> bool:
    """True if the request was still running or queued (it ends TPM_ECANCELLED)."""
    return _check(_lib.tpm_server_cancel(s, int(ticket)), ok=(TPM_OK, TPM_NOTFOUND)) == TPM_OK


def tpm_server_stats_get(s) -> dict:
    st = tpm_server_stats()
    _check(_lib.tpm_server_stats_get(s, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in tpm_server_stats._fields_}


def tpm_server_destroy(s) -> None:
    _lib.tpm_server_destroy(s)


KERNEL_KINDS = {0: "level2", 1: "middle", 2: "last", 3: "step"}


def tpm_profile_enable(on: bool) -> None:
    _check(_lib.tpm_profile_enable(1 if on else 0))


def tpm_profile_read(max_items: int = 4096):
    out = (tpm_kernel_time * max_items)()
    n = ctypes.c_int32(0)
    _check(_lib.tpm_profile_read(out, int(max_items), ctypes.byref(n)))
    return [{"kind": KERNEL_KINDS[out[i].kind], "level": out[i].level,
             "chunk_points": out[i].chunk_points, "ms": out[i].ms} for i in range(n.value)]


# ------------------------------------------------------------------ owners
class Graph:
    def __init__(self, n, src, dst, tau, color, num_colors, tile_edges=0, tile_held=0,
                 transit=None, delay=None, undirected=False):
        self.n = int(n)
        self.m = int(len(src)) * (2 if undirected else 1)
        self.h = tpm_graph_create(n, src, dst, tau, color, num_colors,
                                  TPM_UNDIRECTED if undirected else 0, tile_edges, tile_held,
                                  transit, delay)

    @classmethod
    def from_temporal(cls, g, **kw):
        return cls(g.n, g.src, g.dst, g.tau, g.color, g.num_colors, **kw)

    def stats(self) -> dict:
        return tpm_graph_stats_get(self.h)

    def sieve(self, multiset, seed, mask=None, chunk=0, loc=False, stream=None, prune=False):
        ids = self.stats()["edge_ids"] if loc else None
        return tpm_sieve(self.h, multiset, seed, mask, chunk, ids, stream, prune)

    def sieve_noalloc(self, multiset, seed, total, per_point=None, error_flags=None, stream=None):
        tpm_sieve_noalloc(self.h, multiset, seed, total, per_point, error_flags, stream)

    def rainbow(self, k, seed=1, reps=1):
        return tpm_rainbow_decide(self.h, k, seed, reps)

    def layer(self, tup) -> "Graph":
        """Layered graph of the ordered colour tuple (VC-PATH-MOTIF)."""
        g = Graph.__new__(Graph)
        g.h = tpm_graph_layer(self.h, tup)
        st = tpm_graph_stats_get(g.h)
        g.n, g.m = st["n"], st["m"]
        return g

    def sd(self, s, d) -> "Graph":
        """(s,d)-COLORFUL-PATH instance: s and d recoloured with num_colors and
        num_colors + 1, s's in-edges and d's out-edges removed.  Sieve it with the
        internal colours plus those two."""
        g = Graph.__new__(Graph)
        g.h = tpm_graph_sd(self.h, s, d)
        st = tpm_graph_stats_get(g.h)
        g.n, g.m = st["n"], st["m"]
        return g

    def static_sieve(self, multiset, seed):
        return tpm_static_sieve(self.h, multiset, seed)

    def prune_static(self, multiset, seed, reps=1) -> "Graph":
        """Preprocessing steps (i) + (ii): the subgraph on the vertices the static
        vertex-localised sieve marks for one of `reps` seeds."""
        g = Graph.__new__(Graph)
        g.h = tpm_graph_prune_static(self.h, multiset, seed, reps)
        st = tpm_graph_stats_get(g.h)
        g.n, g.m = st["n"], st["m"]
        return g

    def vertex_ids(self):
        return tpm_graph_vertex_ids(self.h)

    def prune(self, colors=None, times=None) -> "Graph":
        """Subgraph on the edges whose endpoints both have a colour in `colors` and
        whose timestamp is in `times` (None: no restriction); same vertex ids,
        colours and input edge ids."""
        g = Graph.__new__(Graph)
        g.h = tpm_graph_prune(self.h, colors, times)
        st = tpm_graph_stats_get(g.h)
        g.n, g.m = st["n"], st["m"]
        return g

    def decide(self, multiset, seed, reps=1) -> bool:
        return tpm_decide(self.h, multiset, seed, reps)

    def extract(self, multiset, seed, max_reps=8):
        return tpm_extract(self.h, multiset, seed, max_reps)

    def extract_ex(self, multiset, seed, max_reps=8, method=0):
        return tpm_extract_ex(self.h, multiset, seed, max_reps, method)

    def extract_optimum(self, multiset, seed, reps=4, method=0):
        return tpm_extract_optimum(self.h, multiset, seed, reps, method)

    def batch(self, queries, chunk=0, use_graph=False, prune=False, streams=0, per_point=False):
        return tpm_batch_run(self.h, queries, chunk, use_graph, prune, streams, per_point)

    def sieve_vertex(self, multiset, seed, mask=None):
        return tpm_sieve_vertex(self.h, multiset, seed, mask)

    def time_buckets(self, multiset, seed):
        return tpm_time_buckets(self.h, multiset, seed)

    def optimum_time(self, multiset, seed, reps=1) -> int:
        return tpm_optimum_time(self.h, multiset, seed, reps)

    def retile(self, tile_edges) -> None:
        tpm_graph_retile(self.h, tile_edges)

    def autotune(self, k, seed=1) -> dict:
        return tpm_autotune(self.h, k, seed)

    def close(self, _destroy=_lib.tpm_graph_destroy):
        # the library call is bound at definition: at interpreter exit the module's
        # globals may already be gone when a graph is collected
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Server:
    """Owner of a serving loop over a resident graph (tpm_server_*)."""

    def __init__(self, graph: Graph, state_bytes=0, max_lanes=0, extract_paths=0,
                 prune_queries=0, streams=0):
        self.graph = graph
        self.h = tpm_server_create(graph.h, state_bytes, max_lanes, extract_paths, prune_queries,
                                   streams)
        self._pp = {}  # ticket -> per-point buffer the server writes

    def submit(self, multiset, seed, want_path=0, per_point=False, deadline_ms=0.0) -> int:
        """per_point=True: the polled result carries the uint8[2^k] per-point values."""
        buf = np.zeros(1 << len(multiset), dtype=np.uint8) if per_point else None
        t = tpm_server_submit(self.h, multiset, seed, want_path, buf, deadline_ms)
        if buf is not None:
            self._pp[t] = buf
        return t

    def cancel(self, ticket) -> bool:
        return tpm_server_cancel(self.h, ticket)

    def stats(self) -> dict:
        return tpm_server_stats_get(self.h)

    def poll(self, max_results=64):
        res = tpm_server_poll(self.h, max_results)
        for r in res:
            buf = self._pp.pop(r["ticket"], None)
            if buf is not None and r["status"] == TPM_OK:
                r["per_point"] = buf
        return res

    def drain(self, n, timeout_s=600.0):
        """Poll until n results arrived (or raise on timeout)."""
        import time
        got, t0 = [], time.monotonic()
        while len(got) < n:
            got += self.poll(256)
            if len(got) < n:
                if time.monotonic() - t0 > timeout_s:
                    raise TimeoutError(f"{len(got)} of {n} results after {timeout_s}s")
                time.sleep(0.001)
        return got

    def close(self, _destroy=_lib.tpm_server_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
