#!/usr/bin/env python3
"""EMST throughput on one MI355X.

One step = one emst_build of the whole synthetic cloud (tree construction,
every Boruvka round, canonical edge order), points resident in HBM before
the timed region starts.  The default workload is the 37M-point
cosmology-like cloud (the paper's headline 37M 3D workload, Section 4).
Prints one JSON line:

  value         Mpoints/s over the K timed steps (n * K / seconds)
  roofline      the traversal kernel (the dominant kernel), against 8 TB/s
                HBM.  achieved = the bytes the launch must bring from HBM
                at least once (every node record it loads, once, plus the
                fixed bytes of every query) / average launch duration (HIP
                events on the library's stream, live in this run); traffic
                = HBM bytes the counters measured per launch; logical = the
                bytes of every record examination as if none were cached
  cpu_baseline  the CPU oracle (kd-tree Boruvka, OpenMP on the host cores
                this run may use) on the same cloud, also the parity check;
                plus one thread on a stated sample
  batched       512 clouds in one emst_build_batched vs one emst_build per
                cloud (same GPU, resident inputs)
  serving       Poisson request stream: continuous batching vs one request
                per launch (FIFO) and the round-granular solver, p50/p99

Bytes per unit (3D; 2D in brackets):
  node record      64 [48] B, plus 8 B of child labels after the first round
  per query        4*dim + 16 B  (own coordinates, label, bound, candidate)
  logical: internal child 8*dim + 8 B, leaf child 4*dim + 8 B
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EMST Mpoints/sec at 1 GPU + HBM roofline fraction; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0

# Measured HBM traffic of the traversal kernel: rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs (KiB per dispatch, averaged over the uninstrumented
# traversal launches of one build), scaled by what the same counters read for
# a plain 1 GiB device copy (FETCH_SIZE 0.5x, WRITE_SIZE 1.0x of the bytes the
# copy moves, so factors 2.0 and 1.0).  Keyed by workload, traversal variant
# and a hash of the traversal sources: once the kernel changes there is no
# entry and `traffic` is null until the counters are taken again.
TRAFFIC_SOURCES = ("traverse.h", "emst_common.h", "emst_kernels.h")
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0
MEASURED_TRAFFIC = {
    # (workload, variant, source hash): (FETCH_SIZE KiB, WRITE_SIZE KiB, TCC hit fraction, profile)
    ("cosmology3d_37m", 13, "a2025fcf28faa80d"):
        (1172456.2, 294876.0, 0.881, "profiles/k_traverse_fast_cosmology3d_37m.md"),
    ("clustered3d_2m", 13, "a2025fcf28faa80d"):
        (70849.3, 18651.3, 0.878, "profiles/k_traverse_fast_clustered3d_2m.md"),
}
# What bounds the traversal, from counters of the same runs (per launch
# type): VALU busy = VALU issue cycles / (SIMDs x kernel cycles), lane
# utilisation = active lanes per VALU instruction / 64, resident waves per
# CU, scalar instructions per vector instruction.
MEASURED_LIMITER = {
    # (workload, variant, source hash): {"full": {...}, "list": {...}, "profile": path}
    ("cosmology3d_37m", 13, "a2025fcf28faa80d"): {
        "bound_by": "instruction issue x lane divergence (not HBM)",
        "full": {"launches": "rounds 0-1", "valu_busy": 0.568, "lane_utilisation": 0.406,
                 "salu_per_valu": 0.94, "waves_per_cu": 27.2, "of_waves_per_cu": 32, "l2_hit": 0.907,
                 "hbm_frac": 0.098},
        "list": {"launches": "rounds 2-10", "valu_busy": 0.415, "lane_utilisation": 0.532,
                 "salu_per_valu": 1.00, "waves_per_cu": 24.7, "of_waves_per_cu": 32, "l2_hit": 0.854,
                 "hbm_frac": 0.150},
        "profile": "profiles/k_traverse_fast_cosmology3d_37m.md",
    },
    ("clustered3d_2m", 13, "a2025fcf28faa80d"): {
        "bound_by": "instruction issue x lane divergence (not HBM)",
        "full": {"launches": "rounds 0-1", "valu_busy": 0.511, "lane_utilisation": 0.403,
                 "salu_per_valu": 0.94, "waves_per_cu": 23.8, "of_waves_per_cu": 32, "l2_hit": 0.914,
                 "hbm_frac": 0.083},
        "list": {"launches": "rounds 2-8", "valu_busy": 0.291, "lane_utilisation": 0.566,
                 "salu_per_valu": 0.99, "waves_per_cu": 15.3, "of_waves_per_cu": 32, "l2_hit": 0.828,
                 "hbm_frac": 0.111},
        "profile": "profiles/k_traverse_fast_clustered3d_2m.md",
    },
}


def traversal_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2207_00514_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def logical_bytes(dim: int, queries: int, internal: int, leaf: int) -> int:
    return internal * (8 * dim + 8) + leaf * (4 * dim + 8) + queries * (4 * dim + 16)


def unique_bytes(dim: int, rnd: int, queries: int, touched: int) -> int:
    rec = (64 if dim == 3 else 48) + (0 if rnd == 0 else 8)  # the first round derives labels
    return touched * rec + queries * (4 * dim + 16)


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def same_tree(a, b) -> bool:
    import numpy as np
    return (np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
            and np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32)))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cosmology3d_37m",
                    choices=["uniform2d_10k", "clustered3d_2m", "cosmology3d_37m", "skewed3d_2m", "batched512", "serving"])
    ap.add_argument("--legs", default="batched,serving",
                    help="extra legs of the single-cloud run, comma-separated from {batched, serving}, or 'none'")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per measured run")
    ap.add_argument("--serve-warmup", type=int, default=100, help="serving: warm-up requests")
    ap.add_argument("--serve-workers", type=int, default=4,
                    help="serving: worker streams of the continuous-batching server")
    ap.add_argument("--n", type=int, default=None, help="resize the workload (same recipe)")
    ap.add_argument("--variant", type=int, default=None, help="traversal variant (default: library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=None)
    ap.add_argument("--serial-sample", type=int, default=500_000,
                    help="points of the one-thread oracle sample (the cloud's first points; it is shuffled)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--sweep", type=str, default=None,
                    help="comma-separated sizes: EMST throughput of the workload's recipe at every size "
                         "(size scaling), each checked against the oracle within --sweep-oracle-budget")
    ap.add_argument("--sweep-oracle-budget", type=float, default=240.0,
                    help="seconds of oracle time the sweep may spend on parity")
    ap.add_argument("--mreach", type=str, default=None,
                    help="comma-separated k_pts: time core distances and the mutual-reachability MST "
                         "(HDBSCAN*) on the workload instead of the EMST")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        return 2

    if args.mreach:
        return bench_mreach(args)
    if args.sweep:
        return bench_sweep(args)
    if args.workload == "batched512":
        res = batched_leg(args)
        line = {"metric": METRIC, "value": res["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": res["ms"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "batched512", "clouds": res["clouds"], "points": res["points"], "seed": 4},
                "batched": res}
        print(json.dumps(line), flush=True)
        ok = res["equals_solo"] and res.get("oracle_sample_parity", True) and res["captured_rounds"]["equal_results"]
        return 0 if ok else 1
    if args.workload == "serving":
        res = serving_leg(args)
        b9 = res["0.9"]["batched"]
        line = {"metric": METRIC, "value": round(b9["mpoints_per_s"], 3), "unit": "Mpoints/s", "n_gpus": 1,
                "steps": args.requests, "warmup": args.serve_warmup, "ms_per_step": round(b9["mean_ms"], 3),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                "data": "synthetic", "config": {"workload": "serving", "requests": args.requests, "seed": 5},
                "serving": res}
        print(json.dumps(line), flush=True)
        return 0 if res["results_equal"] else 1
    return bench_single(args)


def bench_single(args) -> int:
    import numpy as np
    import torch

    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import workloads as W

    t_start = time.perf_counter()
    spec = W.WORKLOADS[args.workload]
    log(f"generating {args.workload}")
    pts_np = W.make(args.workload, args.n)
    n, dim = pts_np.shape
    log(f"generated n={n} in {time.perf_counter() - t_start:.1f} s")
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(pts_np).to(dev)
    m = n - 1
    out = (torch.empty((m, 2), dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.float32, device=dev),
           torch.empty(m, dtype=torch.float32, device=dev))
    ctx = emst.Context(0)
    if args.variant is not None:
        ctx.set_traversal(args.variant)
    ctx.workspace(n, dim)
    torch.cuda.synchronize()

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # instrumented (untimed) run: children examined and records touched per round
    ctx.set_counting(True)
    ctx.build(pts, out=out)
    torch.cuda.synchronize()
    cst = ctx.stats()
    ctx.set_counting(False)

    ctx.set_profiling(True)
    for _ in range(args.warmup):
        ctx.build(pts, out=out)
    torch.cuda.synchronize()

    trav_ms = 0.0
    launches = 0
    phases = {"tree_ms": 0.0, "rounds_ms": 0.0, "finalize_ms": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trav_round = None  # per round, the shortest traversal launch of the timed steps
    for _ in range(args.steps):
        ctx.build(pts, out=out)
        st = ctx.stats()
        trav_ms += st["traversal_ms"]
        launches += st["rounds"]
        for k in phases:
            phases[k] += st[k]
        tr = list(st["traversal_ms_round"][:st["rounds"]])
        trav_round = tr if trav_round is None else [min(a, b) for a, b in zip(trav_round, tr)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    ms_per_step = 1e3 * secs / args.steps
    value = n * args.steps / secs / 1e6
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} Mpoints/s")

    rounds = cst["rounds"]
    q_round, t_round = cst["queries_round"], cst["records_touched_round"]
    uniq = [unique_bytes(dim, r, q, t) for r, (q, t) in enumerate(zip(q_round, t_round))]
    logi = [logical_bytes(dim, q, ci, li)
            for q, ci, li in zip(q_round, cst["child_tests_round"], cst["leaf_tests_round"])]
    avg_launch_ms = trav_ms / max(launches, 1)
    sec_launch = avg_launch_ms * 1e-3
    uniq_launch = sum(uniq) / max(rounds, 1)
    logi_launch = sum(logi) / max(rounds, 1)
    achieved = uniq_launch / sec_launch / 1e9 if avg_launch_ms > 0 else 0.0
    logical_rate = logi_launch / sec_launch / 1e9 if avg_launch_ms > 0 else 0.0
    variant_ran = int(st["traversal_variant"])
    src_hash = traversal_source_hash()
    key = (args.workload, variant_ran, src_hash)
    meas = None if args.n is not None else MEASURED_TRAFFIC.get(key)
    lim = None if args.n is not None else MEASURED_LIMITER.get(key)
    traffic = None if meas is None else int(meas[0] * 1024 * FETCH_FACTOR + meas[1] * 1024 * WRITE_FACTOR)
    queries = max(sum(q_round), 1)

    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_frac": None if traffic is None else round(traffic / sec_launch / 1e9 / HBM_PEAK_GBS, 4),
        "kernel": "k_traverse_lane" if variant_ran == 0 else "k_traverse_fast",
        "variant": variant_ran,
        "source_hash": src_hash,
        "avg_launch_ms": round(avg_launch_ms, 4),
        "launches_per_step": rounds,
        "algorithmic_bytes_per_launch": int(uniq_launch),
        "algorithmic_bytes": "node records loaded in the launch, each once (64 B + 8 B of child labels after "
                             "the first round), plus 4*dim + 16 B per query",
        "records_touched_per_launch": int(sum(t_round) / max(rounds, 1)),
        "logical": {"bytes_per_launch": int(logi_launch), "rate_gbs": round(logical_rate, 1),
                    "rate_frac": round(logical_rate / HBM_PEAK_GBS, 4),
                    "cache_served": None if traffic is None else round(1.0 - traffic / logi_launch, 4)},
        "l2_hit": None if meas is None else meas[2],
        "traffic_profile": None if meas is None else meas[3],
        "limiter": lim,
        "children_examined_per_query_round": round((cst["child_tests"] + cst["leaf_tests"]) / queries, 2),
        "dist_evals_per_query_round": round(cst["dist_evals"] / queries, 2),
    }

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": int(n), "dim": int(dim), "seed": spec["seed"],
                   "traversal_variant": args.variant if args.variant is not None else "default"},
        "mfeatures_per_s": round(value * dim, 3),
        "rounds": rounds,
        "phases_ms_per_step": {k: round(v / args.steps, 4) for k, v in phases.items()},
        "roofline": roofline,
        # per Borůvka round: the counting run's components, queries, tests per
        # query and node records loaded; the shortest traversal launch of the
        # timed steps (HIP events)
        "round_table": [
            {"round": r, "components": int(cst["components"][r]), "queries": int(q_round[r]),
             "child_tests_per_query": round(cst["child_tests_round"][r] / max(q_round[r], 1), 2),
             "leaf_tests_per_query": round(cst["leaf_tests_round"][r] / max(q_round[r], 1), 2),
             "records_loaded": int(t_round[r]),
             "traversal_ms_min": None if trav_round is None or r >= len(trav_round) else round(trav_round[r], 3)}
            for r in range(rounds)],
    }
    edges, w, d2 = (t.cpu().numpy() for t in out)
    del ctx, out
    torch.cuda.empty_cache()

    legs = [x for x in args.legs.split(",") if x and x != "none"] if args.n is None else []
    ok = True
    if "batched" in legs:
        line["batched"] = batched_leg(args)
        ok = (ok and line["batched"]["equals_solo"] and line["batched"].get("oracle_sample_parity", True)
              and line["batched"]["captured_rounds"]["equal_results"])
    if "serving" in legs:
        line["serving"] = serving_leg(args)
        ok = ok and line["serving"]["results_equal"]

    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or host_threads()
        log(f"oracle on the whole cloud, {threads} threads")
        c0 = time.perf_counter()
        ref = oracle.kdboruvka(pts_np, threads=threads)
        c1 = time.perf_counter()
        parity = (np.array_equal(edges, ref.edges) and np.array_equal(d2.view(np.uint32), ref.d2.view(np.uint32))
                  and np.array_equal(w.view(np.uint32), ref.w.view(np.uint32)))
        log(f"oracle {c1 - c0:.1f} s, parity {'bit-exact' if parity else 'MISMATCH'}")
        del ref
        ns = min(args.serial_sample, n)
        sample = np.ascontiguousarray(pts_np[:ns])
        s0 = time.perf_counter()
        oracle.kdboruvka(sample, threads=1)
        s1 = time.perf_counter()
        log(f"serial oracle sample {ns} points {s1 - s0:.1f} s")
        line["cpu_baseline"] = {
            "value": round(n / (c1 - c0) / 1e6, 4),
            "unit": "Mpoints/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"the whole {args.workload} cloud (n={n}), one run of kd-tree Boruvka with {threads} "
                      f"OpenMP threads, {c1 - c0:.2f} s (the same run checks parity)",
            "host_cpus": os.cpu_count(),
            "cpu_model": cpu_model(),
            "serial": {"value": round(ns / (s1 - s0) / 1e6, 4), "unit": "Mpoints/s", "cores": 1,
                       "sample": f"the first {ns} points of the same cloud (a uniform random subset: the "
                                 f"cloud is shuffled), kd-tree Boruvka on one thread, {s1 - s0:.2f} s"},
        }
        line["parity"] = "bit-exact" if parity else "MISMATCH"
        ok = ok and parity
    log(f"done in {time.perf_counter() - t_start:.1f} s")
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


def batched_leg(args) -> dict:
    """512 clouds (log-uniform 1e3..2e5 points, half 2D uniform, half 3D
    mixtures): one batched pass vs one emst_build per cloud, same GPU and
    resident inputs."""
    import numpy as np
    import torch

    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import autotune
    from paper_2207_00514_amd import workloads as W

    t_leg = time.perf_counter()
    clouds = W.batched_clouds()
    sizes = [len(c) for c in clouds]
    dims = [c.shape[1] for c in clouds]
    total = sum(sizes)
    dev = torch.device("cuda:0")
    flat = torch.from_numpy(np.concatenate([c.reshape(-1) for c in clouds])).to(dev)
    per = [torch.from_numpy(c).to(dev) for c in clouds]
    ctx = emst.Context(0)
    ctx.workspace(max(sizes), 3)
    ctx.build_batched_flat(flat, sizes, dims)  # sizes the batched workspace
    torch.cuda.synchronize()
    # autotune the traversal shape on this batch (untimed; every candidate
    # gives the same trees), then time the automatic choice
    ms = {}
    for shape in autotune.BATCHED_CANDIDATES:
        autotune._set_shape(ctx, shape)
        ms[shape] = 1e3 * autotune._median_seconds(lambda: ctx.build_batched_flat(flat, sizes, dims), 2)
    best = min(ms, key=ms.get)
    ctx.set_autotune(autotune.table_json([{"mode": "batched", "dim": 3, "n_min": 0, "variant": int(best[0]),
                                           "lds_depth": int(best[1])}]))
    autotune._set_shape(ctx, (-1, 0))
    steps = max(args.steps, 3)
    for _ in range(max(args.warmup, 1)):
        ctx.build_batched_flat(flat, sizes, dims)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.build_batched_flat(flat, sizes, dims)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / steps
    # A/B: the rounds from the third on as replays of a captured graph of two
    # rounds (emst_set_graphs), same inputs and shape
    ctx.set_graphs(True)
    for _ in range(max(args.warmup, 1)):
        ctx.build_batched_flat(flat, sizes, dims)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gout = ctx.build_batched_flat(flat, sizes, dims)
    torch.cuda.synchronize()
    t_graphs = (time.perf_counter() - t0) / steps
    ctx.set_graphs(False)
    graphs_same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
                      for a, b in zip(out, gout))
    del gout
    ctx1 = emst.Context(0)
    ctx1.workspace(max(sizes), 3)
    for c in per[:8]:
        ctx1.build(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solo = [ctx1.build(c) for c in per]
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
               for a, b in zip(out, solo))
    res = {
        "workload": "batched512", "clouds": len(clouds), "points": int(total), "seed": 4,
        "value": round(total / t_batched / 1e6, 3), "unit": "Mpoints/s", "ms": round(t_batched * 1e3, 3),
        "steps": steps,
        "one_cloud_per_launch": {"value": round(total / t_solo / 1e6, 3), "unit": "Mpoints/s",
                                 "ms": round(t_solo * 1e3, 3)},
        "speedup": round(t_solo / t_batched, 2),
        "equals_solo": bool(same),
        "captured_rounds": {"ms": round(t_graphs * 1e3, 3), "eager_ms": round(t_batched * 1e3, 3),
                            "equal_results": bool(graphs_same)},
        "autotuned_shape": {"variant": int(best[0]), "lds_depth": int(best[1])},
        "autotune_ms": {autotune._label(k): round(v, 3) for k, v in ms.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or host_threads()
        rng = np.random.default_rng(0)
        pick = sorted(rng.choice(len(clouds), 16, replace=False).tolist())
        ok = True
        for c in pick:
            ref = oracle.emst(clouds[c], threads=threads)
            got = tuple(x.cpu().numpy() for x in out[c])
            ok = ok and same_tree(got, (ref.edges, ref.w, ref.d2))
        res["oracle_sample_parity"] = bool(ok)
        res["oracle_sample"] = f"clouds {pick} against the oracle (every cloud: tests/test_gpu_parity.py)"
    del ctx, ctx1, flat, per, out, solo
    torch.cuda.empty_cache()
    log(f"batched leg: {res['ms']} ms batched, {res['one_cloud_per_launch']['ms']} ms one per launch, "
        f"{time.perf_counter() - t_leg:.1f} s")
    return res


def serving_leg(args) -> dict:
    """Poisson stream of 3D requests (lognormal sizes, median 5e4, sigma 1.2,
    clipped to [5e3, 4e6]; uniform or clustered).  The continuous-batching
    server (batch granularity, emst_build_batched) and the round-granular
    native solver (emst_solver_*) are compared with a one-request-per-launch
    FIFO server (emst_build per request) on the same arrival trace at 0.5 and
    0.9 of the batched saturation rate.  Every request's result must be the
    same in every server."""
    import numpy as np
    import xxhash

    from paper_2207_00514_amd import serve
    from paper_2207_00514_amd import workloads as W

    t_leg = time.perf_counter()
    count, nwarm = args.requests, args.serve_warmup
    sizes = W.request_sizes(count + nwarm, seed=5)
    clouds = [W.request_cloud(int(n), seed=5000 + i) for i, n in enumerate(sizes)]
    warm, clouds = clouds[:nwarm], clouds[nwarm:]
    log(f"serving: {count} requests, {sum(len(c) for c in clouds)} points generated "
        f"in {time.perf_counter() - t_leg:.1f} s")

    def digest(r):
        if r.error is not None:
            return None
        h = xxhash.xxh3_64()
        for a in (r.edges, r.weights, r.d2):
            h.update(np.ascontiguousarray(a).view(np.uint8))
        return h.intdigest()

    def make(kind, nw):
        if kind == "batched":
            return serve.Server(workers=nw, max_batch=64, budget_bytes=16 << 30)
        if kind == "solver":
            return serve.SolverServer(budget_bytes=16 << 30, max_slots=256)
        return serve.FifoServer()

    def run(kind, rate, reqs):
        srv = make(kind, args.serve_workers)
        rq = [serve.Request(i, c) for i, c in enumerate(reqs)]
        if rate is None:
            arr = [0.0] * len(rq)
        else:
            gaps = np.random.default_rng(7).exponential(1.0 / rate, len(rq))
            arr = list(np.cumsum(gaps) - gaps[0])
        span = serve.replay(srv, rq, arr)
        summ = serve.summary(rq, span)
        dig = [digest(r) for r in rq]
        del rq, srv
        return summ, dig

    for kind in ("batched", "solver", "fifo"):  # warm-up (kernels, allocator)
        run(kind, None, warm)
    # saturated requests/s: the better of two bursts of the whole trace
    bursts = [run("batched", None, clouds)[0] for _ in range(2)]
    mu = max(b["requests"] / b["makespan_s"] for b in bursts)
    res = {"requests": count, "warmup_requests": nwarm, "seed": 5, "workers": args.serve_workers,
           "saturation_qps": round(mu, 1)}
    ok = True
    for frac in (0.5, 0.9):
        lam = frac * mu
        b, db = run("batched", lam, clouds)
        sv, ds = run("solver", lam, clouds)
        f, df = run("fifo", lam, clouds)
        same = db == ds == df and None not in db
        ok = ok and same
        res[f"{frac}"] = {"qps": round(lam, 1), "batched": b, "round_granular_solver": sv,
                          "fifo_one_per_launch": f, "results_equal": same}
        log(f"serving at {frac} mu ({lam:.0f} req/s): batched p50/p99 {b['p50_ms']:.1f}/{b['p99_ms']:.1f} ms, "
            f"solver {sv['p50_ms']:.1f}/{sv['p99_ms']:.1f}, fifo {f['p50_ms']:.1f}/{f['p99_ms']:.1f}")
    res["results_equal"] = ok
    res["p50_ms"] = round(res["0.9"]["batched"]["p50_ms"], 3)
    res["p99_ms"] = round(res["0.9"]["batched"]["p99_ms"], 3)
    log(f"serving leg {time.perf_counter() - t_leg:.1f} s")
    return res


def bench_sweep(args) -> int:
    """EMST time and Mpoints/s of one workload recipe over a range of sizes
    (the saturation size and the linear regime of one GPU), each size checked
    against the oracle while the oracle's time budget lasts; sizes past it
    are marked parity unpinned."""
    import numpy as np
    import torch
    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import workloads as W

    if args.workload in ("batched512", "serving"):
        print("bench.py: --sweep runs on a single-cloud workload", file=sys.stderr)
        return 2
    ctx = emst.Context(0)
    ctx.set_profiling(True)
    threads = args.cpu_threads or host_threads()
    budget = 0.0 if args.no_cpu_baseline else args.sweep_oracle_budget
    rate = None  # oracle points per second seen so far (smallest rate)
    rows = []
    ok = True
    for n in [int(float(x)) for x in args.sweep.split(",")]:
        pts_np = W.make(args.workload, n)
        pts = torch.from_numpy(pts_np).cuda()
        out = None
        for _ in range(args.warmup):
            out = ctx.build(pts, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = ctx.build(pts, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = ctx.stats()
        row = {"n": n, "ms": round(1e3 * dt, 3), "mpoints_per_s": round(n / dt / 1e6, 3),
               "rounds": st["rounds"], "tree_ms": round(st["tree_ms"], 3),
               "rounds_ms": round(st["rounds_ms"], 3), "finalize_ms": round(st["finalize_ms"], 3)}
        est = None if rate is None else n * 1.2 / rate
        if budget > 0 and (est is None or est <= budget):
            import oracle
            got = tuple(t.cpu().numpy() for t in out)
            c0 = time.perf_counter()
            ref = oracle.emst(pts_np, threads=threads)
            c1 = time.perf_counter()
            budget -= c1 - c0
            r = n / max(c1 - c0, 1e-6)
            rate = r if rate is None else min(rate, r)
            par = same_tree(got, (ref.edges, ref.w, ref.d2))
            ok = ok and par
            row["parity"] = "bit-exact" if par else "MISMATCH"
            row["oracle_s"] = round(c1 - c0, 2)
        else:
            row["parity"] = "parity unpinned (oracle time budget)"
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del pts, out
        torch.cuda.empty_cache()
    line = {
        "metric": "EMST Mpoints/sec at 1 GPU over sizes", "value": max(r["mpoints_per_s"] for r in rows),
        "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "sweep": [r["n"] for r in rows]}, "sizes": rows,
        "oracle_threads": threads,
    }
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


def bench_mreach(args) -> int:
    """Mutual-reachability MST (Section 4): per k_pts, the time of the core
    distances alone (T_core) and of the whole MST including them (T_emst),
    both from device-resident points, and parity with the oracle (core
    distances by a kd-tree k-nearest search, tree by kd-Boruvka) unless
    --no-cpu-baseline."""
    import numpy as np
    import torch
    import paper_2207_00514_amd as emst
    from paper_2207_00514_amd import workloads as W

    if args.workload in ("batched512", "serving"):
        print("bench.py: --mreach runs on a single-cloud workload", file=sys.stderr)
        return 2
    pts_np = W.make(args.workload, args.n) if args.n else W.make(args.workload)
    n, dim = pts_np.shape
    pts = torch.from_numpy(pts_np).cuda()
    ctx = emst.Context(0)
    rows = []
    ok = True
    for k in [int(x) for x in args.mreach.split(",")]:
        def timed(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / args.steps
        t_core = timed(lambda: ctx.core_distances(pts, k))
        t_mst = timed(lambda: ctx.build_mreach(pts, k))
        e, w, d2, core2 = ctx.build_mreach(pts, k)
        row = {"k_pts": k, "t_core_ms": round(1e3 * t_core, 3), "t_emst_ms": round(1e3 * t_mst, 3),
               "mpoints_per_s": round(n / t_mst / 1e6, 3)}
        if not args.no_cpu_baseline:
            import oracle
            threads = args.cpu_threads or host_threads()
            c0 = time.perf_counter()
            ref, rcore = oracle.mreach_mst(pts_np, k, threads=threads)
            c1 = time.perf_counter()
            par = (np.array_equal(core2.cpu().numpy().view(np.uint32), rcore.view(np.uint32))
                   and np.array_equal(e.cpu().numpy(), ref.edges)
                   and np.array_equal(d2.cpu().numpy().view(np.uint32), ref.d2.view(np.uint32)))
            row["cpu_oracle_s"] = round(c1 - c0, 2)
            row["parity"] = "bit-exact" if par else "MISMATCH"
            ok = ok and par
        rows.append(row)
    line = {
        "metric": "mutual-reachability MST Mpoints/sec at 1 GPU (T_core, T_emst per k_pts)",
        "value": rows[0]["mpoints_per_s"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": int(n), "dim": int(dim), "metric": "mutual_reachability"},
        "k_pts": rows,
    }
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
