#!/usr/bin/env python3
"""Throughput of the GF(2^8) temporal path-motif sieve on one MI355X.

One step = one full sieve query (all 2^k sieve points, levels 2..k, XOR reduction)
through the C ABI, on the k = 10 directed Chung-Lu workload (n = 1e6, m = 1e8,
beta = 2.5, timestamps U[1, 1e4], 16 colours, a multiset of 10 i.i.d. colours).
The graph index is built before timing (inputs resident in HBM).

Prints one JSON line: edge-updates/s (m * k * 2^k per query), per-query latency,
the roofline of the dominant kernel (measured with HIP events on its stream) and
the CPU oracle timed on a bounded sample of the same workload.  The default run adds
two objects, each with its own graph and an oracle spot check: "batched" (256 queries
of uneven k on n = 2e6, m = 1e8: one at a time versus the batched forms) and "serving"
(a stream prefix against n = 1e7, m = 1e9: capacity and p50/p99 latency per mode).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GF(2^8) sieve edge-updates/s (m·k·2^k) at k=10; HBM GB/s; p50/p99 query ms"
HBM_PEAK_GBPS = 8000.0
# committed rocprofv3 PMC summaries of the middle-level kernel, by sieve points per row
PMC_FILES = {1024: os.path.join(ROOT, "profiles", "k10_level_middle_pmc.txt"),
             256: os.path.join(ROOT, "profiles", "k10_narrow_c256_middle_pmc.txt"),
             64: os.path.join(ROOT, "profiles", "k10_narrow_c64_middle_pmc.txt"),
             32: os.path.join(ROOT, "profiles", "k10_narrow_c32_middle_pmc.txt"),
             16: os.path.join(ROOT, "profiles", "k10_narrow_c16_middle_pmc.txt")}
KERNEL_SRC = os.path.join(ROOT, "paper_2001_07158_amd", "csrc", "tpm_sieve.hip")


def kernel_hash(points: int = 1024) -> str:
    """Hash of the level kernel's source for rows of `points` sieve points: the file up
    to the narrow-row kernel (1024-point rows: parameters, helpers, k_level), or up to
    the end of the narrow-row kernel (smaller rows)."""
    text = open(KERNEL_SRC, "rb").read()
    marker = b"// Narrow rows:" if points >= 1024 else b"__global__ void k_prep"
    cut = text.find(marker)
    return hashlib.sha256(text if cut < 0 else text[:cut]).hexdigest()[:16]


def read_traffic(points: int):
    """HBM bytes per launch of the middle-level kernel from committed rocprofv3 PMC
    summaries, if they were taken on the current kernel source at this row width."""
    path = PMC_FILES.get(points)
    if path is None or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    if kv.get("kernel_hash") != kernel_hash(points):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="k10",
                    choices=["k10", "k5", "tiny", "batched", "serving", "preproc"])
    ap.add_argument("--queries", type=int, default=0,
                    help="batched/serving: number of queries (default 256 / 120)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="batched/serving: shrink n and m (1.0 = the named workload)")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving: arrival rate as a fraction of the measured capacity")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--tile-edges", type=int, default=0, help="work tile size of the index (0 = default)")
    ap.add_argument("--autotune", action="store_true",
                    help="batched: time the tile/chunk candidates first and apply the fastest")
    ap.add_argument("--cpu-points", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pruned", action="store_true",
                    help="skip the colour-pruned comparison run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the decide / extraction / optimum-time timings")
    ap.add_argument("--prune", action="store_true",
                    help="serving: run each request alone on the subgraph of its colours")
    ap.add_argument("--no-extract", action="store_true",
                    help="serving: decide only (default: extract a path on every hit)")
    ap.add_argument("--no-batched", action="store_true",
                    help="default run: skip the batched workload")
    ap.add_argument("--no-serving", action="store_true",
                    help="default run: skip the serving workload")
    ap.add_argument("--serve-queries-pruned", type=int, default=120,
                    help="serving: stream prefix of the pruned mode")
    ap.add_argument("--serve-queries-row", type=int, default=16,
                    help="serving: stream prefix of the row mode")
    ap.add_argument("--serve-spot", type=int, default=2,
                    help="serving: served requests checked against the oracle")
    ap.add_argument("--row-only", action="store_true", help="serving: the row mode only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for profiler counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sieve's "
              "multi-GPU form (sieve points sharded, one XOR exchange) is not built.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2001_07158_amd import tpm
    from synth import CONFIGS, make_config_graph, make_config_query

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "preproc":
        return bench_preproc(args)

    cfg = CONFIGS[args.workload]
    t_gen = time.perf_counter()
    g = make_config_graph(args.workload)
    M = make_config_query(args.workload)
    k = len(M)
    t_gen = time.perf_counter() - t_gen
    print(f"# workload {args.workload}: n={g.n} m={g.m} k={k} M={list(M)} (generated in "
          f"{t_gen:.1f}s)", file=sys.stderr, flush=True)

    t_idx = time.perf_counter()
    G = tpm.Graph.from_temporal(g, tile_edges=args.tile_edges)
    st = G.stats()
    t_idx = time.perf_counter() - t_idx
    print(f"# index built in {t_idx:.2f}s: rows={st['rows']} tiles={st['tiles']} "
          f"slots={st['slots']} gathers={st['gathers']} segments={st['segments']}",
          file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    seed0 = 20010715
    for w in range(args.warmup):
        G.sieve(M, seed0 + 1000 + w, chunk=args.chunk, stream=stream)
        print(f"# warmup {w} done", file=sys.stderr, flush=True)

    tpm.tpm_profile_read()  # drain
    tpm.tpm_profile_enable(True)
    lat = []
    per_point = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        pp, tot = G.sieve(M, seed0 + s, chunk=args.chunk, stream=stream)
        lat.append((time.perf_counter() - ts) * 1e3)
        if s == 0:
            per_point = pp
        print(f"# step {s}: {lat[-1]:.1f} ms total={tot}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tpm.tpm_profile_enable(False)
    ktimes = tpm.tpm_profile_read()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    units = float(g.m) * k * (1 << k)
    value = units / (ms_per_step / 1e3)
    chunk_pts = ktimes[0]["chunk_points"] if ktimes else min(1 << k, 1024)

    # ---- roofline of the dominant kernel (middle levels; level 2 when k == 3)
    kinds = {}
    for t in ktimes:
        kinds.setdefault(t["kind"], []).append(t["ms"])
    dom = "middle" if "middle" in kinds else ("level2" if "level2" in kinds else "last")
    avg_ms = float(np.mean(kinds[dom])) if dom in kinds else float("nan")
    C = chunk_pts
    struct = 16.0 * g.m + 12.0 * st["tiles"] + float(st["segments"]) * C
    # level 2 (k >= 3) from coefficients: a k-byte XOR scan over the positions (two passes
    # reading dst, src and edge id, 24 bytes a position, and the row index; W and V written
    # per row, 20 bytes) once a query, then per chunk the expansion (W, V and the z row of
    # a row read, 36 bytes, the row written)
    l2_scan = 28.0 * g.m + 20.0 * st["rows"]
    l2_rows = (float(C) + 36.0) * st["rows"]
    if dom == "middle":
        alg = (st["gathers"] + st["rows"]) * float(C) + struct
    elif dom == "level2":
        alg = l2_rows
    else:
        alg = st["gathers"] * float(C) + struct
    achieved = alg / (avg_ms / 1e3) / 1e9
    # each read request to HBM moves a 128-byte line on this GPU (rocprofv3: a 1 GiB
    # streaming read issues 2^23 TCC_EA0_RDREQ), so a random gather of a row shorter than
    # 128 bytes moves 128 bytes: the least traffic a launch can have
    line_b = 128.0
    if dom == "middle":
        xfer = st["gathers"] * max(float(C), line_b) + st["rows"] * float(C) + struct
    elif dom == "level2":
        xfer = l2_rows
    else:
        xfer = st["gathers"] * max(float(C), line_b) + struct
    traffic = read_traffic(C) if dom == "middle" else None
    # whole-query algorithmic bytes (all levels, all chunks)
    nchunks = max(1, (1 << k) // C)
    q_bytes = l2_scan + nchunks * (l2_rows
                                   + max(0, k - 3) * ((st["gathers"] + st["rows"]) * float(C) + struct)
                                   + (st["gathers"] * float(C) + struct))
    hbm_alg = q_bytes / (ms_per_step / 1e3) / 1e9

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: directed Chung-Lu n={g.n} m={g.m} beta=2.5 "
                         f"t=[1,{cfg['t']}] q={cfg['q']} k={k}") if cfg["kind"] == "chung_lu"
            else f"{args.workload}: uniform n={g.n} m={g.m} t=[1,{cfg['t']}] q={cfg['q']} k={k}",
            "k": k, "n": g.n, "m": g.m, "sieve_points": 1 << k, "chunk_points": C,
            "rows_stored": st["rows"], "tiles": st["tiles"],
        },
        "query_ms_p50": float(np.percentile(lat, 50)),
        "query_ms_p99": float(np.percentile(lat, 99)),
        "hbm_gbps_algorithmic_query": hbm_alg,
        # the DP's own count: k - 1 edge levels per point (the metric counts k)
        "edge_level_updates_per_s": float(g.m) * (k - 1) * (1 << k) / (ms_per_step / 1e3),
        "copy_gbps_reference": copy_gbps(torch),
        "roofline": {
            "bound": "hbm",
            "kernel": (f"k_level ({C}-point rows, {dom} level)" if C >= 1024
                       else f"k_slot ({C}-point rows, {dom} level)" if C >= 128
                       else f"k_narrow ({C}-point rows, {dom} level)"),
            "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
            "alg_bytes_per_launch": alg, "avg_launch_ms": avg_ms, "launches": len(kinds.get(dom, [])),
            # the same with every gather charged at least one 128-byte line (rows of
            # fewer than 128 points): achieved and fraction of peak on that count
            "min_transfer_bytes_per_launch": xfer,
            "achieved_min_transfer": xfer / (avg_ms / 1e3) / 1e9,
            "frac_min_transfer": xfer / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
            "kernel_hash": kernel_hash(C),
        },
        "cpu_baseline": None,
    }

    # ---- decide, witness extraction and the optimum timestamp for the same query
    # (outside the timed region): extraction is the sieve with localisation, then k-2
    # smaller sieves restricted to one in-list each
    if not args.no_extras:
        torch.cuda.synchronize()
        te = time.perf_counter()
        found = G.decide(M, seed0, reps=1)
        t_dec = (time.perf_counter() - te) * 1e3
        te = time.perf_counter()
        rc, verts, edges, n_ext = G.extract_ex(M, seed0, max_reps=8, method=0)
        t_ext = (time.perf_counter() - te) * 1e3
        ok = rc == tpm.TPM_OK  # the library verifies every path it returns
        e1 = None
        if k <= 6:  # the paper's self-reducibility needs O(k log n) decisions
            te = time.perf_counter()
            rc1, _, _, n1 = G.extract_ex(M, seed0, max_reps=4, method=1)
            e1 = {"ms": (time.perf_counter() - te) * 1e3, "sieves": n1,
                  "found": rc1 == tpm.TPM_OK}
        # the paper's vertex-localisation extraction: one localised sieve, then a
        # reverse temporal DFS from a certified end vertex
        te = time.perf_counter()
        rc2, _, _, n2 = G.extract_ex(M, seed0, max_reps=4, method=2)
        e2 = {"ms": (time.perf_counter() - te) * 1e3, "sieves": n2, "found": rc2 == tpm.TPM_OK}
        te = time.perf_counter()
        t_opt_val = G.optimum_time(M, seed0, reps=1)
        t_opt = (time.perf_counter() - te) * 1e3
        line["extras"] = {
            "decide_ms": t_dec, "found": bool(found), "extract_ms": t_ext,
            "extract_sieves": n_ext, "extract_over_decide": t_ext / t_dec,
            "path_verified": bool(ok), "extract_selfreduce": e1, "extract_vertexloc": e2,
            "optimum_time_ms": t_opt, "optimum_time": t_opt_val,
        }
        print(f"# vertex-localisation extraction: {e2}", file=sys.stderr, flush=True)
        print(f"# decide {t_dec:.1f} ms, extract {t_ext:.1f} ms (path ok={ok}), optimum time "
              f"{t_opt_val} in {t_opt:.1f} ms", file=sys.stderr, flush=True)

    # ---- the same query on the colour-pruned graph (the paper's preprocessing step (i):
    # edges whose endpoints both have a colour of M); outside the timed region and
    # reported beside `value`, which stays the unpruned sweep
    if not args.no_pruned:
        cols = sorted(set(int(c) for c in M))
        tp, tq, same, m_kept = [], [], True, 0
        for r in range(3):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            Gp = G.prune(cols)
            tb = time.perf_counter()
            ppp, _ = Gp.sieve(M, seed0, chunk=args.chunk, stream=stream)
            torch.cuda.synchronize()
            tc_ = time.perf_counter()
            same &= bool(np.array_equal(ppp, per_point))
            m_kept = Gp.m
            Gp.close()
            tp.append((tb - ta) * 1e3)
            tq.append((tc_ - tb) * 1e3)
        tot_ms = float(np.median(np.array(tp) + np.array(tq)))
        line["pruned"] = {
            "colours": cols, "m_kept": m_kept, "prune_ms": float(np.median(tp)),
            "query_ms": float(np.median(tq)), "total_ms": tot_ms,
            "speedup_vs_unpruned": ms_per_step / tot_ms, "per_point_equal": same,
            "edge_updates_per_s_in_unpruned_units": units / (tot_ms / 1e3),
        }
        print(f"# pruned: m_kept={m_kept} prune {np.median(tp):.1f} ms + query "
              f"{np.median(tq):.1f} ms, equal={same}", file=sys.stderr, flush=True)

        # preprocessing step (ii) on top: the static vertex-localised sieve over the
        # arcs between vertices of M's colours, then the subgraph on the vertices it
        # marks for one of 3 seeds (a vertex of a match is missed by one GF(2^8) sieve
        # with probability about 1/256, by all three about 6e-8); with every match kept
        # the query total is the unpruned one
        reps = 3
        torch.cuda.synchronize()
        ta = time.perf_counter()
        sv = G.static_sieve(M, seed0)
        tb = time.perf_counter()
        Gs = G.prune_static(M, seed0, reps=reps)
        tc_ = time.perf_counter()
        _, tot_s = Gs.sieve(M, seed0, chunk=args.chunk, stream=stream)
        torch.cuda.synchronize()
        td = time.perf_counter()
        line["static_prefilter"] = {
            "static_sieve_ms": (tb - ta) * 1e3, "reps": reps,
            "prune_ms": (tc_ - tb) * 1e3,  # static instance + reps sieves + subgraph
            "query_ms": (td - tc_) * 1e3, "n_kept_one_seed": int((sv != 0).sum()), "m_kept": Gs.m,
            "total_equal": bool(tot_s == int(np.bitwise_xor.reduce(per_point))),
        }
        Gs.close()
        print(f"# static prefilter: sieve {(tb - ta) * 1e3:.1f} ms, prune {(tc_ - tb) * 1e3:.1f} ms, "
              f"n_kept={int((sv != 0).sum())} m_kept={line['static_prefilter']['m_kept']}, "
              f"query {(td - tc_) * 1e3:.1f} ms", file=sys.stderr, flush=True)

    if args.copy_calibration:
        calibration_kernels()

    if not args.no_cpu_baseline:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        rng = np.random.default_rng(7)
        P = min(args.cpu_points, 1 << k)
        pts = np.sort(rng.choice(1 << k, P, replace=False)).astype(np.uint32)
        t_oi = time.perf_counter()
        idx = oracle.Index(g)
        t_oi = time.perf_counter() - t_oi
        print(f"# oracle index {t_oi:.1f}s; evaluating {P} points on {nthreads} threads",
              file=sys.stderr, flush=True)
        tc = time.perf_counter()
        want = idx.eval(M, seed0, pts, nthreads=nthreads)
        tc = time.perf_counter() - tc
        parity = bool(np.array_equal(per_point[pts], want))
        line["cpu_baseline"] = {
            "value": float(g.m) * k * P / tc, "unit": "edge-updates/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{P} of {1 << k} sieve points over the full graph, all levels "
                      f"({tc:.1f}s; index build {t_oi:.1f}s not timed)",
            "parity_on_sample": parity,
        }
        print(f"# oracle sample parity: {parity}", file=sys.stderr, flush=True)

    G.close()
    del g
    # the batched and serving workloads, each with its own graph (outside the timed
    # region of `value`)
    ok = True
    if args.workload == "k10" and not args.no_batched:
        line["batched"] = run_batched(args)
        ok &= line["batched"]["all_forms_equal_alone"] and line["batched"]["oracle_spot_check"]["equal"]
    if args.workload == "k10" and not args.no_serving:
        line["serving"] = run_serving(args)
        ok &= line["serving"]["modes_equal"] and line["serving"]["oracle_spot_check"]["equal"]
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


def calibration_kernels() -> None:
    """Kernels of known size for scaling the profiler's traffic counters: a 1 GiB device
    copy (reads and writes 1 GiB) and the library's 1 GiB streaming read."""
    import torch
    from paper_2001_07158_amd import tpm

    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    o = torch.zeros(1, dtype=torch.int64, device="cuda")
    tpm.tpm_stream_read(a, a.numel(), o, torch.cuda.current_stream())
    torch.cuda.synchronize()
    del a, b, o
    torch.cuda.empty_cache()


def copy_gbps(torch) -> float:
    """Device-to-device copy rate (bytes read + written per second, GB/s) of a 4 GiB
    buffer: the streaming reference beside the kernel's roofline figures."""
    a = torch.empty(1 << 32, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 32) / (ms / 1e3) / 1e9


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _spot_check(g, samples, seed_of, per_point_of, max_points=16, nthreads=0):
    """Oracle per-point values for a sample of queries, against the GPU's: each query on
    an oracle index of the edges between vertices of its own colours (exact: other
    vertices have z = 0), all points for k <= 6, else max_points random points."""
    import numpy as np
    import oracle

    t0 = time.perf_counter()
    rng = np.random.default_rng(99)
    rows, ok = [], True
    for ms in samples:
        k = len(ms)
        pts = (np.arange(1 << k, dtype=np.uint32) if k <= 6 else
               np.sort(rng.choice(1 << k, max_points, replace=False)).astype(np.uint32))
        idx = oracle.Index(g, keep_colours=set(int(c) for c in ms))
        want = idx.eval(ms, seed_of(ms), pts, nthreads=nthreads)
        got = per_point_of(ms)
        same = got is not None and bool(np.array_equal(got[pts], want))
        ok &= same
        rows.append({"k": k, "points": int(pts.size), "edges_indexed": idx.m, "equal": same})
        del idx
    return {"equal": bool(ok), "queries": rows, "seconds": time.perf_counter() - t0}


def run_batched(args, nq=None, spot=True) -> dict:
    """256 queries of uneven size k ~ U{3..10} against one resident Chung-Lu graph
    (n = 2e6, m = 1e8): one at a time through tpm_sieve (plain launches, the whole
    graph), then tpm_batch_run in packed rows (uneven k side by side, plain launches
    and HIP-graph replay) and with each query on its colour subgraph (several at once on
    their own streams).  Every batched per-point byte must equal the same query run
    alone; a sample of queries is checked against the CPU oracle."""
    import numpy as np
    import torch
    from paper_2001_07158_amd import tpm
    from synth import CONFIGS, make_config_graph, make_config_query

    cfg = CONFIGS["batched"]
    nq = nq or args.queries or cfg["nq"]
    t_gen = time.perf_counter()
    g = make_config_graph("batched", scale=args.scale)
    qs = [{"multiset": [int(c) for c in make_config_query("batched", i)],
           "seed": 20010715 + 7919 * i} for i in range(nq)]
    ks = [len(q["multiset"]) for q in qs]
    _log(f"# batched: n={g.n} m={g.m} queries={nq} k-histogram={np.bincount(ks).tolist()} "
         f"(generated in {time.perf_counter() - t_gen:.1f}s)")
    G = tpm.Graph.from_temporal(g)
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = G.autotune(max(ks), seed=1)
        tuned["seconds"] = time.perf_counter() - t0
        _log(f"# autotune: tile_edges={tuned['tile_edges']} chunk={tuned['chunk']} "
             f"({tuned['seconds']:.1f}s)")
    st = G.stats()
    # warm-up: one query of each size through every form
    warm = [qs[ks.index(k)] for k in sorted(set(ks))]
    for q in warm:
        G.sieve(q["multiset"], q["seed"])
    G.batch(warm)
    G.batch(warm, use_graph=True)
    G.batch(warm, prune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [G.sieve(q["multiset"], q["seed"])[0] for q in qs]
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    _log(f"# one at a time: {t_alone:.2f}s")
    forms = {}
    for name, kw in (("packed", {}), ("packed_graph_replay", {"use_graph": True}),
                     ("pruned_streams", {"prune": True}),
                     ("pruned_one_stream", {"prune": True, "streams": 1})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = G.batch(qs, per_point=True, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        same = all(np.array_equal(r["per_point"], a) for r, a in zip(res, alone))
        forms[name] = {"seconds": t, "qps": nq / t, "speedup_vs_one_at_a_time": t_alone / t,
                       "per_point_equal_alone": bool(same),
                       "found": int(sum(r["found"] for r in res))}
        _log(f"# {name}: {t:.2f}s ({nq / t:.1f} queries/s), per-point equal alone: {same}")
    best = max(forms, key=lambda f: forms[f]["qps"])
    units = float(sum(g.m * k * (1 << k) for k in ks))
    out = {
        "metric": "batched queries/s (k ~ U{3..10}), GF(2^8) sieve",
        "value": forms[best]["qps"], "unit": "queries/s", "best_form": best,
        "one_at_a_time_qps": nq / t_alone, "speedup_vs_one_at_a_time": forms[best]["qps"] * t_alone / nq,
        "forms": forms,
        "edge_updates_per_s_best": units / forms[best]["seconds"],
        "edge_updates_per_s_one_at_a_time": units / t_alone,
        "config": {"workload": f"batched: directed Chung-Lu n={g.n} m={g.m} beta=2.5 "
                               f"t=[1,{cfg['t']}] q={cfg['q']}, {nq} queries k~U{{3..10}}",
                   "rows_stored": st["rows"], "tile_edges": st["tile_edges"]},
        "autotune": tuned,
    }
    G.close()
    if spot:
        # the smallest and the largest k, and two in between: per-point bytes of the
        # batched run (equal to the alone run above) against the oracle
        order = sorted(range(nq), key=lambda i: (ks[i], i))
        pick = sorted(set([order[0], order[len(order) // 3], order[2 * len(order) // 3], order[-1]]))
        by_ms = {tuple(qs[i]["multiset"]): i for i in pick}
        out["oracle_spot_check"] = _spot_check(
            g, [qs[i]["multiset"] for i in pick],
            lambda ms: qs[by_ms[tuple(ms)]]["seed"], lambda ms: alone[by_ms[tuple(ms)]])
        out["oracle_spot_check"]["query_indices"] = pick
        _log(f"# batched oracle spot check: {out['oracle_spot_check']}")
    out["all_forms_equal_alone"] = all(f["per_point_equal_alone"] for f in forms.values())
    return out


def bench_batched(args) -> int:
    if args.copy_calibration:
        calibration_kernels()
    line = run_batched(args)
    line.update({"n_gpus": 1, "higher_is_better": True, "dtype": "u8", "data": "synthetic"})
    print(json.dumps(line), flush=True)
    ok = line["all_forms_equal_alone"] and line.get("oracle_spot_check", {}).get("equal", True)
    return 0 if ok else 1


def _serve(srv, qs, rate=None, log_every=20.0):
    """Submits every query of qs: all at once (closed-loop burst, rate None) or with
    Poisson arrivals at `rate` queries/s; returns (results by query index, seconds from
    the first submission to the last result)."""
    import numpy as np

    ticket_of, got = {}, {}

    def take(res):
        for r in res:
            got[ticket_of[r["ticket"]]] = r

    gaps = (np.zeros(len(qs)) if rate is None
            else np.random.default_rng(17).exponential(1.0 / rate, len(qs)))
    t0 = time.perf_counter()
    t_last = t0
    next_t = t0
    for i, q in enumerate(qs):
        next_t += gaps[i]
        while time.perf_counter() < next_t:
            take(srv.poll(256))
            time.sleep(0.0003)
        ticket_of[srv.submit(q["multiset"], q["seed"], per_point=True)] = i
        if time.perf_counter() - t_last > log_every:
            _log(f"#   submitted {i + 1}, {len(got)} results")
            t_last = time.perf_counter()
    while len(got) < len(qs):
        take(srv.poll(256))
        if time.perf_counter() - t_last > log_every:
            _log(f"#   {len(got)} of {len(qs)} results")
            t_last = time.perf_counter()
        time.sleep(0.0005)
    return got, time.perf_counter() - t0


def run_serving(args, modes=("pruned", "pruned_single", "row"), spot=True) -> dict:
    """A Poisson stream of queries (k ~ U{3..10}, 16 colours) against a resident
    Chung-Lu graph (n = 1e7, m = 1e9) through the serving loop, with a path extracted
    on every hit: capacity from a closed-loop burst of the whole stream prefix (and,
    apart, of its first third), then arrivals at `load` x capacity; queries/s delivered
    and p50/p99 latency (submit to result, host clock).  Modes: "pruned" (each request on the subgraph of
    its colours; a second, express worker holds short requests, and the device is lent
    to them between two levels of a long sieve), "pruned_single" (the same with one
    worker: requests one after the other) and "row" (one resident multi-query row over
    the whole graph, continuous batching at level granularity).
    Results of a request must be the same in every mode and equal the oracle."""
    import numpy as np
    from paper_2001_07158_amd import tpm
    from synth import CONFIGS, make_config_graph, make_config_query

    cfg = CONFIGS["serving"]
    t_gen = time.perf_counter()
    g = make_config_graph("serving", scale=args.scale)
    _log(f"# serving: n={g.n} m={g.m} generated in {time.perf_counter() - t_gen:.1f}s")
    t_idx = time.perf_counter()
    G = tpm.Graph.from_temporal(g)
    st = G.stats()
    t_idx = time.perf_counter() - t_idx
    _log(f"# index: rows={st['rows']} tiles={st['tiles']} built in {t_idx:.1f}s")
    out = {"metric": "serving queries/s and p50/p99 latency (Poisson arrivals), GF(2^8) sieve",
           "extract_on_hit": not args.no_extract, "load": args.load,
           "config": {"workload": f"serving: directed Chung-Lu n={g.n} m={g.m} beta=2.5 "
                                  f"t=[1,{cfg['t']}] q={cfg['q']}, stream k~U{{3..10}}",
                      "rows_stored": st["rows"], "index_build_s": t_idx},
           "modes": {}}
    nmax = max(args.queries or 0, args.serve_queries_pruned, args.serve_queries_row)
    qs = [{"multiset": [int(c) for c in make_config_query("serving", i)],
           "seed": 90001 + 7919 * i} for i in range(nmax)]
    per_point = {}
    for mode in modes:
        pruned = mode.startswith("pruned")
        nq = args.queries or (args.serve_queries_pruned if pruned else args.serve_queries_row)
        srv = tpm.Server(G, prune_queries=1 if pruned else 0,
                         extract_paths=0 if args.no_extract else 1,
                         streams=1 if mode == "pruned_single" else 0)
        # warm-up: two requests
        for q in qs[:2]:
            srv.submit(q["multiset"], q["seed"])
        srv.drain(2)
        # capacity: the whole prefix as one closed-loop burst; then the same prefix again
        # with Poisson arrivals at load x capacity.  First, a burst of the prefix's first
        # third alone (a lighter part of the stream: a second, smaller measure)
        n3 = max(1, nq // 3)
        _, t_third = _serve(srv, qs[:n3])
        _log(f"# serving mode {mode}: {nq} queries as a burst, then Poisson at {args.load} x capacity")
        burst, t_burst = _serve(srv, qs[:nq])
        cap = nq / t_burst
        rate = args.load * cap
        got, t_open = _serve(srv, qs[:nq], rate=rate)
        sstats = srv.stats()
        srv.close()
        lat_open = np.array([got[i]["t_done_ms"] - got[i]["t_submit_ms"] for i in range(nq)])
        hits = [r for r in list(burst.values()) + list(got.values()) if r["found"]]
        paths_ok = (int(sum(r["path_status"] == tpm.TPM_OK for r in hits))
                    if not args.no_extract else None)
        bad = [i for i in range(nq) if got[i]["status"] != tpm.TPM_OK or burst[i]["status"] != tpm.TPM_OK]
        for res in (burst, got):
            for i in range(nq):
                if res[i]["status"] != tpm.TPM_OK:
                    continue
                if i in per_point:
                    per_point[i]["modes_equal"] &= bool(np.array_equal(per_point[i]["pp"],
                                                                       res[i]["per_point"]))
                else:
                    per_point[i] = {"pp": res[i]["per_point"], "modes_equal": True}
        ks = np.array([len(q["multiset"]) for q in qs[:nq]])
        out["modes"][mode] = {
            "value": cap, "unit": "queries/s (closed-loop capacity)",
            "capacity_qps_closed_loop": cap, "arrival_rate_qps": rate,
            "capacity_qps_first_third": n3 / t_third, "first_third_queries": n3,
            "delivered_qps_open_loop": nq / t_open,
            "latency_ms_p50": float(np.percentile(lat_open, 50)),
            "latency_ms_p99": float(np.percentile(lat_open, 99)),
            "latency_ms_p50_by_k": {int(k): float(np.percentile(lat_open[ks == k], 50))
                                    for k in sorted(set(ks.tolist()))},
            "stream_prefix": nq, "found": len(hits), "paths_ok": paths_ok, "failed": len(bad),
            "server_stats": sstats,
        }
        _log(f"# {mode}: capacity {cap:.2f} q/s (first third {n3 / t_third:.2f}); at {rate:.2f} q/s: "
             f"{nq / t_open:.2f} q/s delivered, "
             f"p50 {np.percentile(lat_open, 50):.0f} ms, p99 {np.percentile(lat_open, 99):.0f} ms, "
             f"hits {len(hits)}, paths ok {paths_ok}, trims {sstats.get('trims')}")
    G.close()
    out["modes_equal"] = all(v["modes_equal"] for v in per_point.values())
    # headline: the library's default serving mode (pruned, with an express worker)
    head = "pruned" if "pruned" in out["modes"] else next(iter(out["modes"]))
    out["headline_mode"] = head
    out["best_capacity_mode"] = max(out["modes"], key=lambda md: out["modes"][md]["capacity_qps_closed_loop"])
    out["value"] = out["modes"][head]["capacity_qps_closed_loop"]
    out["unit"] = "queries/s (closed-loop capacity); latency at load x capacity"
    out["latency_ms_p50"] = out["modes"][head]["latency_ms_p50"]
    out["latency_ms_p99"] = out["modes"][head]["latency_ms_p99"]
    if spot:
        # the served requests with the fewest distinct colours (smallest colour
        # subgraphs, so the oracle finishes in seconds): every point against the oracle
        cand = sorted(per_point, key=lambda i: (len(set(qs[i]["multiset"])), len(qs[i]["multiset"]), i))
        pick = cand[:args.serve_spot]
        by_ms = {tuple(qs[i]["multiset"]): i for i in pick}
        out["oracle_spot_check"] = _spot_check(
            g, [qs[i]["multiset"] for i in pick], lambda ms: qs[by_ms[tuple(ms)]]["seed"],
            lambda ms: per_point[by_ms[tuple(ms)]]["pp"])
        out["oracle_spot_check"]["query_indices"] = pick
        _log(f"# serving oracle spot check: {out['oracle_spot_check']}")
    return out


def bench_serving(args) -> int:
    line = run_serving(args, modes=("pruned", "pruned_single") if args.prune else ("row",)
                       if args.row_only else ("pruned", "pruned_single", "row"))
    line.update({"n_gpus": 1, "higher_is_better": True, "dtype": "u8", "data": "synthetic"})
    print(json.dumps(line), flush=True)
    ok = line["modes_equal"] and line.get("oracle_spot_check", {}).get("equal", True)
    return 0 if ok else 1


def bench_preproc(args) -> int:
    """The paper's preprocessing / vertex-localisation experiment on its own kind of
    input: random 20-regular undirected graphs (configuration model), t = 100, k = 8,
    n = 1e2 .. 1e5.  PATH-MOTIF: 30 colours, a random multiset of 8; COLORFUL-PATH: 8
    colours, the multiset {0..7}.  Extraction time (median over instances) with the
    self-reducibility method, with preprocessing step (ii) first (3 seeds), with the
    vertex-localisation method, and with both."""
    import numpy as np
    from paper_2001_07158_amd import tpm
    from synth import regular_graph

    d, t, k = 20, 100, 8
    ninst = 3
    rows = []
    for problem, q in (("PATH-MOTIF", 30), ("COLORFUL-PATH", k)):
        for n in (100, 1_000, 10_000, 100_000):
            res = {"algebraic": [], "pre": [], "vloc": [], "pre+vloc": []}
            found = {key: 0 for key in res}
            m_kept = []
            for inst in range(ninst):
                seed = 1000 * n + 17 * inst + (0 if problem == "PATH-MOTIF" else 7)
                g = regular_graph(n, d, t, q, seed)
                rng = np.random.default_rng(seed)
                M = ([int(c) for c in rng.integers(0, q, k)] if problem == "PATH-MOTIF"
                     else list(range(k)))
                G = tpm.Graph(g.n, g.src, g.dst, g.tau, g.color, q, undirected=True)
                G.extract_ex(M, 1, max_reps=2, method=2)  # warm-up
                for key in res:
                    t0 = time.perf_counter()
                    H = G
                    if key.startswith("pre"):
                        H = G.prune_static(M, seed, reps=3)
                        if key == "pre":
                            m_kept.append(H.m)
                    rc = H.extract_ex(M, seed, max_reps=4, method=2 if key.endswith("vloc") else 1)[0]
                    res[key].append((time.perf_counter() - t0) * 1e3)
                    found[key] += rc == tpm.TPM_OK
                    if H is not G:
                        H.close()
                G.close()
            row = {"problem": problem, "n": n, "m_undirected": n * d // 2, "instances": ninst,
                   "m_arcs_after_pre_median": float(np.median(m_kept)),
                   **{f"{key}_ms": float(np.median(v)) for key, v in res.items()},
                   "found": found}
            row["speedup_pre"] = row["algebraic_ms"] / row["pre_ms"]
            row["speedup_vloc"] = row["algebraic_ms"] / row["vloc_ms"]
            row["speedup_pre_vloc"] = row["algebraic_ms"] / row["pre+vloc_ms"]
            rows.append(row)
            _log(f"# {problem} n={n}: " + ", ".join(f"{key} {row[key + '_ms']:.1f} ms" for key in res)
                 + f", arcs after (ii) {row['m_arcs_after_pre_median']:.0f} of {n * d}, found {found}")
    line = {"metric": "extraction ms with preprocessing step (ii) and vertex localisation (k = 8)",
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "preproc: random 20-regular undirected graphs, t = 100, k = 8"},
            "rows": rows}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
