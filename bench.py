#!/usr/bin/env python3
"""Throughput of the GF(2^8) temporal path-motif sieve on one MI355X.

One step = one full sieve query (all 2^k sieve points, levels 2..k, XOR reduction)
through the C ABI, on the k = 10 directed Chung-Lu workload (n = 1e6, m = 1e8,
beta = 2.5, timestamps U[1, 1e4], 16 colours, a multiset of 10 i.i.d. colours).
The graph index is built before timing (inputs resident in HBM).

Prints one JSON line: edge-updates/s (m * k * 2^k per query), per-query latency,
the roofline of the dominant kernel (measured with HIP events on its stream) and
the CPU oracle timed on a bounded sample of the same workload.
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
             256: os.path.join(ROOT, "profiles", "k10_narrow_c256_middle_pmc.txt")}
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
    if dom == "middle":
        alg = (st["gathers"] + st["rows"]) * float(C) + struct
    elif dom == "level2":
        alg = (g.m + st["rows"]) * float(C) + struct
    else:
        alg = st["gathers"] * float(C) + struct
    achieved = alg / (avg_ms / 1e3) / 1e9
    traffic = read_traffic(C) if dom == "middle" else None
    # whole-query algorithmic bytes (all levels, all chunks)
    nchunks = max(1, (1 << k) // C)
    q_bytes = nchunks * ((g.m + st["rows"]) * float(C) + struct
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
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

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

    print(json.dumps(line), flush=True)
    G.close()
    return 0


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


def bench_batched(args) -> int:
    """256 queries of uneven size k ~ U{3..10} against one resident Chung-Lu graph
    (n = 2e6, m = 1e8): one query at a time through tpm_sieve versus tpm_batch_run;
    every batched total must equal the same query run alone."""
    import numpy as np
    import torch
    from paper_2001_07158_amd import tpm
    from synth import CONFIGS, make_config_graph, make_config_query

    cfg = CONFIGS["batched"]
    nq = args.queries or cfg["nq"]
    g = make_config_graph("batched", scale=args.scale)
    qs = [{"multiset": [int(c) for c in make_config_query("batched", i)],
           "seed": 20010715 + 7919 * i} for i in range(nq)]
    ks = [len(q["multiset"]) for q in qs]
    _log(f"# batched: n={g.n} m={g.m} queries={nq} k-histogram={np.bincount(ks).tolist()}")
    G = tpm.Graph.from_temporal(g)
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = G.autotune(max(ks), seed=1)
        tuned["seconds"] = time.perf_counter() - t0
        _log(f"# autotune: tile_edges={tuned['tile_edges']} chunk={tuned['chunk']} "
             f"({tuned['seconds']:.1f}s)")
    st = G.stats()
    # warm-up: one query of each size both ways
    warm = [qs[ks.index(k)] for k in sorted(set(ks))]
    for q in warm:
        G.sieve(q["multiset"], q["seed"])
    G.batch(warm)
    G.batch(warm, use_graph=True)
    G.batch(warm, prune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = [G.sieve(q["multiset"], q["seed"])[1] for q in qs]
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    _log(f"# one-at-a-time: {t_alone:.2f}s")
    t0 = time.perf_counter()
    res = G.batch(qs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    _log(f"# batched: {t_batch:.2f}s")
    t0 = time.perf_counter()
    res_g = G.batch(qs, use_graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    _log(f"# batched, graph replay: {t_graph:.2f}s")
    t0 = time.perf_counter()
    res_p = G.batch(qs, prune=True)
    torch.cuda.synchronize()
    t_pruned = time.perf_counter() - t0
    _log(f"# each query on its colour subgraph: {t_pruned:.2f}s")
    same = all(r["total"] == a for r, a in zip(res, alone))
    same_g = all(r["total"] == a for r, a in zip(res_g, alone))
    same_p = all(r["total"] == a for r, a in zip(res_p, alone))
    units = float(sum(g.m * k * (1 << k) for k in ks))
    line = {
        "metric": "batched queries/s (256 queries, k ~ U{3..10}), GF(2^8) sieve",
        "value": nq / t_batch, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "one_at_a_time_qps": nq / t_alone, "speedup_vs_one_at_a_time": t_alone / t_batch,
        "edge_updates_per_s_batched": units / t_batch,
        "edge_updates_per_s_one_at_a_time": units / t_alone,
        "graph_replay_qps": nq / t_graph, "graph_replay_totals_equal_alone": same_g,
        "pruned_qps": nq / t_pruned, "pruned_totals_equal_alone": same_p,
        "all_totals_equal_alone": same, "found": int(sum(r["found"] for r in res)),
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batched: directed Chung-Lu n={g.n} m={g.m} beta=2.5 "
                               f"t=[1,{cfg['t']}] q={cfg['q']}, {nq} queries k~U{{3..10}}",
                   "rows_stored": st["rows"], "tile_edges": tuned["tile_edges"] if tuned else None},
        "autotune": tuned,
    }
    print(json.dumps(line), flush=True)
    G.close()
    return 0 if (same and same_g and same_p) else 1


def bench_serving(args) -> int:
    """A Poisson stream of queries (k ~ U{3..10}) against a resident Chung-Lu graph
    (n = 1e7, m = 1e9) through the serving loop: capacity from a closed-loop burst,
    then arrivals at `load` x capacity; queries/s and p50/p99 latency (submit to
    result, host clock)."""
    import numpy as np
    from paper_2001_07158_amd import tpm
    from synth import CONFIGS, make_config_graph, make_config_query

    cfg = CONFIGS["serving"]
    nq = args.queries or 120
    t_gen = time.perf_counter()
    g = make_config_graph("serving", scale=args.scale)
    _log(f"# serving: n={g.n} m={g.m} generated in {time.perf_counter() - t_gen:.1f}s")
    t_idx = time.perf_counter()
    G = tpm.Graph.from_temporal(g)
    st = G.stats()
    _log(f"# index: rows={st['rows']} tiles={st['tiles']} built in {time.perf_counter() - t_idx:.1f}s")
    qs = [{"multiset": [int(c) for c in make_config_query("serving", i)],
           "seed": 90001 + 7919 * i} for i in range(nq)]
    srv = tpm.Server(G, prune_queries=1 if args.prune else 0,
                     extract_paths=0 if args.no_extract else 1)

    def drain(n, got=None):
        """Poll until n results arrived, printing progress every 20 s."""
        got = [] if got is None else got
        t_last = time.perf_counter()
        while len(got) < n:
            got += srv.poll(256)
            if time.perf_counter() - t_last > 20:
                _log(f"# {len(got)} of {n} results")
                t_last = time.perf_counter()
            time.sleep(0.001)
        return got

    # capacity: a closed-loop burst of the first third of the stream
    nb = max(8, nq // 3)
    t0 = time.perf_counter()
    for q in qs[:nb]:
        srv.submit(q["multiset"], q["seed"])
    burst = drain(nb)
    cap = nb / (time.perf_counter() - t0)
    _log(f"# capacity {cap:.3f} queries/s from a burst of {nb}")
    # open loop: Poisson arrivals at load x capacity for the rest of the stream
    rate = args.load * cap
    rng = np.random.default_rng(17)
    gaps = rng.exponential(1.0 / rate, nq - nb)
    t_start = time.perf_counter()
    next_t = t_start
    results = []
    t_last = t_start
    for i, q in enumerate(qs[nb:]):
        next_t += gaps[i]
        while time.perf_counter() < next_t:
            results += srv.poll(256)
            time.sleep(0.0005)
        srv.submit(q["multiset"], q["seed"])
        if time.perf_counter() - t_last > 20:
            _log(f"# submitted {i + 1}, {len(results)} results")
            t_last = time.perf_counter()
    results = drain(nq - nb, results)
    t_total = time.perf_counter() - t_start
    sstats = srv.stats()
    srv.close()
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in results])
    # spot check: a few streamed results against the same query run alone
    by_ticket = {r["ticket"]: r for r in results}
    check = sorted(by_ticket)[:4]
    same = True
    for t in check:
        q = qs[nb + (t - nb - 1)]
        same &= by_ticket[t]["total"] == G.sieve(q["multiset"], q["seed"])[1]
    line = {
        "metric": "serving queries/s and p50/p99 latency (Poisson arrivals), GF(2^8) sieve",
        "value": len(results) / t_total, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
        "capacity_qps_closed_loop": cap, "arrival_rate_qps": rate, "streamed_queries": len(results),
        "burst_queries": nb, "found": int(sum(r["found"] for r in results + burst)),
        "spot_check_equal_alone": bool(same), "dtype": "u8", "data": "synthetic",
        "mode": "per-request colour pruning" if args.prune else "continuous batching (resident row)",
        "extract_on_hit": not args.no_extract,
        "paths_ok": (int(sum(r["path_status"] == tpm.TPM_OK for r in results + burst if r["found"]))
                     if not args.no_extract else None),
        "server_stats": sstats,
        "config": {"workload": f"serving: directed Chung-Lu n={g.n} m={g.m} beta=2.5 "
                               f"t=[1,{cfg['t']}] q={cfg['q']}, stream prefix of {nq} queries "
                               f"k~U{{3..10}}", "rows_stored": st["rows"]},
    }
    print(json.dumps(line), flush=True)
    G.close()
    return 0 if same else 1


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
