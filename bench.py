"""Benchmark: single-source compression + sieve BFS on one MI355X.

A step is one whole search (every level: expand, update, reduction, sieve,
WAH compress, decode/merge) from one root. The default workload is an R-MAT
graph of scale 26 (edgefactor 16, initiator 0.57/0.19/0.19/0.05, ids permuted)
on an 8 x 8 block grid (p = 8), roots drawn by the seeded root picker; K roots
are timed after W warm-up roots. The graph is resident in HBM before timing.

The timed searches run without instrumentation; the same roots are then
searched again with per-kernel HIP events and level statistics for the byte
counts, the time split and the roofline.

Prints one JSON line: harmonic-mean GTEPS over the timed roots (TEPS = input
tuples in the reached component / search time), compression ratios over all
messages, each kernel's roofline against HBM bandwidth (algorithmic bytes
from the level statistics, time from HIP events recorded on the library's
stream; top-down and bottom-up levels apart), the batched comparison (64
roots in one batched search against the same roots one at a time, R-MAT
scale 24), the serving run (Poisson queries over a resident pool of six
graphs: p50/p99 latency and GTEPS, then a saturating burst) and the CPU
oracle on the host's cores, timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

METRIC = "GTEPS (harmonic mean over roots) + message compression ratio; serving p50/p99"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(REPO, "profiles", "expand_traffic.json")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64, help="timed roots")
    ap.add_argument("--warmup", type=int, default=2, help="untimed roots first")
    ap.add_argument("--workload", default="rmat26_p8", help="rmat10_p1 | rmat22_p4 | rmat26_p8")
    ap.add_argument("--alpha", type=float, default=None, help="direction rule alpha (default: the library's)")
    ap.add_argument("--beta", type=float, default=None, help="direction rule beta (default: the library's)")
    ap.add_argument("--no-sieve", action="store_true", help="Alg. 2 messages (no directory)")
    ap.add_argument("--mode", default="auto", choices=["auto", "sparse", "dense", "bottom_up"],
                    help="evaluation of each level's product (results are identical): auto = "
                         "top-down or bottom-up per level; sparse = top-down only")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-cores oracle baseline (0: the host's cores, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-workload", default="rmat24_p4",
                    help="workload of the batched comparison (64 roots in one search)")
    ap.add_argument("--batch-reps", type=int, default=3, help="timed batches")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-qps", type=float, default=2000.0, help="Poisson arrival rate of the serving run")
    ap.add_argument("--serve-requests", type=int, default=4000, help="queries of the serving run")
    ap.add_argument("--serve-slots", type=int, default=4, help="concurrent batched searches")
    ap.add_argument("--serve-burst", type=int, default=2048,
                    help="queries of the saturated run (submitted back to back after the Poisson run)")
    ap.add_argument("--json-out", default=None, help="also write a detailed report here")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy(mib: int):
    """A plain copy kernel of known size: reads and writes mib MiB once each,
    so hardware byte counters taken on it give their scale factor."""
    import torch
    n = mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)


def expand_kernel_hash() -> str:
    path = os.path.join(REPO, "paper_1208_5542_amd", "csrc", "csbfs", "bfs.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def expansion_bytes(s: dict, n: int, p: int) -> int:
    """Algorithmic bytes of expanding one level. Top-down: the column ids of
    every scanned row (4 B), the row-offset pair of every view bit (8 B), one
    pass over the p views and one over the visited bits. Bottom-up: column
    ids read, one row-offset pair per examined vertex, the p views, and the
    visited and live bits scanned for candidates."""
    from paper_1208_5542_amd import csbfs
    if s["direction"] == csbfs.DIR_BOTTOM_UP:
        return 4 * s["edges"] + 8 * s["pulled"] + p * n // 8 + 2 * n // 8
    return 4 * s["edges"] + 8 * s["view_bits"] + p * n // 8 + n // 8


def codec_bytes(s: dict, n: int, p: int) -> tuple[int, int]:
    """Algorithmic bytes of one level's encoder and decoder. Encoder (the
    update that forms f^k fused with the sieve and compression of its
    messages): f_i read once per receiver and V_{j,i} once (2 p n/8), the
    update's visited bits (3 n/8), 8 B (level, degree) per new vertex and
    the stream words written. Decoder: the stream words read and the p
    views written (p n/8)."""
    words = (s["wah_sieved_bytes"] + s["self_bytes"]) // 8
    enc = 2 * p * n // 8 + 3 * n // 8 + 8 * s["frontier"] + 8 * words
    dec = 8 * words + p * n // 8
    return enc, dec


def batched_bytes(s: dict, n: int, p: int, B: int) -> tuple[int, int]:
    """Algorithmic bytes of one batched level: its expansion and its update.
    Top-down expansion: the column ids of every scanned row (4 B) and the
    visit mask of each target (8 B), plus one pass over the B planes of the
    p views. Bottom-up expansion: every vertex's visit mask and row offsets
    (16 B), the column ids read (4 B) and each one's frontier mask (8 B),
    and the B view planes cleared. Update: visit and discovery masks read
    (16 B per vertex), frontier masks written (8 B), degrees read (4 B) and
    the B frontier planes written."""
    from paper_1208_5542_amd import csbfs
    if s["direction"] == csbfs.DIR_BOTTOM_UP:
        exp = 16 * n + 12 * s["edges"] + B * p * n // 8
    else:
        exp = 12 * s["edges"] + B * p * n // 8
    upd = 28 * n + B * n // 8
    return exp, upd


def load_traffic(workload: str):
    """HBM bytes per expansion launch from committed rocprofv3 counter runs,
    only if they were taken on the current expansion kernel source."""
    try:
        with open(COUNTERS) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    ent = d.get(workload)
    if not ent or ent.get("source_hash") != expand_kernel_hash():
        return None
    return ent.get("bytes_per_launch")


_CPU = {}


def _cpu_root(root):
    """One root through the oracle's Algorithm 3 in a forked worker (the
    adjacency and directory are inherited from the parent, read-only)."""
    import oracle
    t = time.perf_counter()
    r = _CPU["adj"].alg3(_CPU["p"], _CPU["V"], int(root), max_levels=256)
    dt = time.perf_counter() - t
    return int(root), dt, oracle.teps_m(_CPU["src"], _CPU["dst"], r.level)


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(n, src, dst, p, roots, workers):
    """The oracle as it stands, on the host's cores: its serial Algorithm 3
    (sieve + WAH streams) on the same graph and roots, one root per process,
    `workers` processes at once (forked after the adjacency is built, so
    they share it). The sample is one root per worker; the aggregate rate is
    the sum of the roots' tuples over the wall time of the parallel run.
    The one-thread rate is the harmonic mean of the same roots' own rates."""
    import multiprocessing as mp

    import oracle
    t0 = time.perf_counter()
    _CPU.update(adj=oracle.Adjacency(n, src, dst), V=oracle.directory(n, p, src, dst).reshape(-1),
                p=p, src=src, dst=dst)
    setup = time.perf_counter() - t0
    sample = [int(r) for r in roots[:workers]]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(processes=len(sample)) as pool:
        res = pool.map(_cpu_root, sample, chunksize=1)
    wall = time.perf_counter() - t0
    _CPU.clear()
    m_tot = sum(m for _, _, m in res)
    one = len(res) / sum(dt / m for _, dt, m in res)
    return {
        "value": round(m_tot / wall / 1e9, 4), "unit": "GTEPS", "cores": len(sample), "kind": "oracle",
        "sample": f"{len(sample)} roots of the same graph, one per process on {len(sample)} host cores at once, "
                  f"each through the oracle's serial Algorithm 3 (level loop with sieve and WAH-64 streams); "
                  f"{wall:.1f} s wall; aggregate = sum of the roots' tuples / wall time; setup (adjacency + "
                  f"directory, {setup:.1f} s) untimed",
        "one_thread_gteps": round(one / 1e9, 4),
        "one_thread_note": "harmonic mean over the same roots of each root's own tuples / its own time",
        "host_cores": host_cores(),
    }


def batched_section(args):
    """64 roots searched together by the batched engine against the same 64
    roots searched one at a time, on one resident graph: aggregate GTEPS
    (sum over roots of the reached component's tuples / time) of both, and
    whether every root's levels agree between the two engines."""
    import torch

    from paper_1208_5542_amd import csbfs, inputs

    wl = inputs.WORKLOADS[args.batched_workload]
    n, p = wl.n, wl.p
    t = time.perf_counter()
    src, dst = wl.tuples()
    roots = [int(r) for r in wl.roots(src, dst, 64)]
    g = csbfs.Graph(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n, p)
    del src, dst
    torch.cuda.synchronize()
    log(f"[bench] batched: graph {wl.name} built in {time.perf_counter() - t:.1f}s")
    B = len(roots)
    beng = csbfs.BatchEngine(g, max_roots=64, max_levels=256)
    seng = csbfs.Engine(g, max_levels=256)
    blevel = torch.empty((B, n), dtype=torch.int32, device="cuda")
    level = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    beng.bfs(roots, blevel)
    seng.bfs(roots[0], level, parent)
    torch.cuda.synchronize()
    bms, bstats = [], None
    for _ in range(max(args.batch_reps, 1)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        res = beng.bfs(roots, blevel, with_stats=False)
        e1.record(stream)
        torch.cuda.synchronize()
        bms.append(e0.elapsed_time(e1))
    # statistics and per-kernel times from one more, instrumented, batch
    bstats = csbfs.BatchEngine(g, max_roots=64, max_levels=256, flags=csbfs.FLAG_TIMING).bfs(roots, blevel).stats
    m = [g.traversed_tuples(blevel[b]) for b in range(B)]
    sms, match = [], True
    for b, r in enumerate(roots):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        seng.bfs(r, level, parent, with_stats=False)
        e1.record(stream)
        torch.cuda.synchronize()
        sms.append(e0.elapsed_time(e1))
        match = match and bool(torch.equal(level, blevel[b]))
    bt = min(bms) / 1e3
    st = sum(sms) / 1e3
    split = {k: round(sum(s[f"ms_{k}"] for s in bstats), 4)
             for k in ("expand", "update", "compress", "decode")}
    raw = sum(s["raw_bytes"] for s in bstats)
    wah = sum(s["wah_sieved_bytes"] for s in bstats)
    out = {
        "workload": wl.name, "scale": wl.scale, "p": p, "roots": B,
        "levels": res.n_levels,
        "batched_ms": round(min(bms), 3), "batched_ms_all": [round(x, 3) for x in bms],
        "batched_gteps": round(sum(m) / bt / 1e9, 4),
        "sequential_ms": round(sum(sms), 3),
        "sequential_gteps": round(sum(m) / st / 1e9, 4),
        "sequential_hmean_gteps": round(B / sum((t / 1e3) / mm for t, mm in zip(sms, m)) / 1e9, 4),
        "speedup": round(st / bt, 3),
        "levels_match_single_root": match,
        "time_split_ms": split,
        "compression_ratio": round(raw / max(wah, 1), 3),
        "edges_scanned": sum(s["edges"] for s in bstats),
    }
    # roofline of the batched kernels (instrumented batch), by direction
    roof = {}
    for name, want in (("expand_top_down", lambda s: s["direction"] != csbfs.DIR_BOTTOM_UP),
                       ("expand_bottom_up", lambda s: s["direction"] == csbfs.DIR_BOTTOM_UP)):
        lv = [s for s in bstats if want(s) and s["ms_expand"] > 0]
        if lv:
            by = sum(batched_bytes(s, n, p, B)[0] for s in lv)
            ms = sum(s["ms_expand"] for s in lv)
            roof[name] = {"levels": len(lv), "bytes": by, "ms": round(ms, 4),
                          "achieved": round(by / (ms / 1e3) / 1e9, 1), "unit": "GB/s",
                          "frac": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    lv = [s for s in bstats if s["ms_update"] > 0]
    if lv:
        by = sum(batched_bytes(s, n, p, B)[1] for s in lv)
        ms = sum(s["ms_update"] for s in lv)
        roof["update"] = {"levels": len(lv), "bytes": by, "ms": round(ms, 4),
                          "achieved": round(by / (ms / 1e3) / 1e9, 1), "unit": "GB/s",
                          "frac": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["roofline"] = roof
    out["levels_by_direction"] = {
        "top_down": sum(1 for s in bstats if s["direction"] != csbfs.DIR_BOTTOM_UP),
        "bottom_up": sum(1 for s in bstats if s["direction"] == csbfs.DIR_BOTTOM_UP)}
    log(f"[bench] batched {out['batched_gteps']} GTEPS vs sequential {out['sequential_gteps']} "
        f"(x{out['speedup']}), levels match: {match}")
    del beng, seng, g
    torch.cuda.empty_cache()
    return out


SERVING_POOL = [("rmat16", 16), ("rmat18", 18), ("rmat20", 20), ("rmat22", 22), ("rmat24", 24), ("er20", 20)]


def serving_section(args):
    """Queries at Poisson arrival times over a resident pool (R-MAT scales
    16-24 and an Erdos-Renyi graph of 2^20 vertices and 8 * 2^20 tuples,
    average degree 16; all on a 4 x 4 grid), each for a uniformly drawn
    graph and root, served by the continuous-batching loop. Latency is
    submit-to-done on the server's clock; GTEPS is the sum over queries of
    the reached component's tuples over the span from the first submit to
    the last completion."""
    import numpy as np
    import torch

    from paper_1208_5542_amd import csbfs, inputs

    t0 = time.perf_counter()
    pool = []
    for name, scale in SERVING_POOL:
        n = 1 << scale
        if name.startswith("er"):
            src, dst = inputs.er_tuples(n, 8 * n, inputs.graph_seed(scale) + 0xE)
        else:
            src, dst = inputs.rmat_tuples(scale, 16)
        g = csbfs.Graph(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n, 4)
        roots = [int(r) for r in inputs.pick_roots(n, src, dst, 128, inputs.graph_seed(scale) + 3)]
        del src, dst
        # traversed tuples per root (TEPS numerator) and the time of the
        # same search on the single-root engine alone, from one search each
        eng = csbfs.Engine(g, max_levels=256)
        level = torch.empty(n, dtype=torch.int32, device="cuda")
        parent = torch.empty(n, dtype=torch.int32, device="cuda")
        eng.bfs(roots[0], level, parent, with_stats=False)
        stream = torch.cuda.current_stream()
        m, ts = [], []
        for r in roots:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            eng.bfs(r, level, parent, with_stats=False)
            e1.record(stream)
            m.append(g.traversed_tuples(level))
            ts.append(e0.elapsed_time(e1) / 1e3)
        del eng, level, parent
        pool.append(dict(name=name, n=n, g=g, roots=roots, m=m, t_single=ts))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"[bench] serving: pool of {len(pool)} graphs ready in {time.perf_counter() - t0:.1f}s")

    budget = 48 << 30
    server = csbfs.Server(slots=args.serve_slots, max_batch=64, max_levels=256, hbm_budget=budget)
    gids = [server.add_graph(e["g"]) for e in pool]
    rng = np.random.default_rng(0x5E5E)
    # warm-up: one batch per graph so engines exist before the timed stream
    for e, gid in zip(pool, gids):
        server.wait(server.submit(gid, e["roots"][0]))
    gaps = rng.exponential(1.0 / args.serve_qps, args.serve_requests)
    picks = [(int(rng.integers(len(pool))), int(rng.integers(128))) for _ in range(args.serve_requests)]
    ids, meta = [], []
    start = time.perf_counter()
    due = start
    for gap, (gi, ri) in zip(gaps, picks):
        due += gap
        delay = due - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(server.submit(gids[gi], pool[gi]["roots"][ri]))
        meta.append((gi, ri))
    infos = [server.wait(i) for i in ids]
    # saturated: a burst submitted back to back, so queues build up and the
    # server batches; its throughput is the pool's capacity
    bpicks = [(int(rng.integers(len(pool))), int(rng.integers(128))) for _ in range(args.serve_burst)]
    bids = [server.submit(gids[gi], pool[gi]["roots"][ri]) for gi, ri in bpicks]
    binfos = [server.wait(i) for i in bids]
    server.close()
    bad = sum(1 for i in infos + binfos if i["status"] != 0)
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos]) * 1e3
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    m_tot = sum(pool[gi]["m"][ri] for gi, ri in meta)
    t_single = sum(pool[gi]["t_single"][ri] for gi, ri in meta)
    per_graph = {}
    for (gi, _), l in zip(meta, lat):
        per_graph.setdefault(pool[gi]["name"], []).append(l)
    out = {
        "pool": [f"{e['name']} (n={e['n']}, p=4)" for e in pool],
        "requests": len(infos), "failed": bad, "offered_qps": args.serve_qps,
        "achieved_qps": round(len(infos) / span, 1),
        "slots": args.serve_slots, "max_batch": 64, "hbm_budget_bytes": budget,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "mean": round(float(lat.mean()), 3), "max": round(float(lat.max()), 3)},
        "latency_p50_ms_by_graph": {k: round(float(np.percentile(v, 50)), 3) for k, v in per_graph.items()},
        "latency_p99_ms_by_graph": {k: round(float(np.percentile(v, 99)), 3) for k, v in per_graph.items()},
        "gteps": round(m_tot / span / 1e9, 4),
        "single_root_gteps_same_requests": round(m_tot / t_single / 1e9, 4),
        "single_root_note": "the same requests searched one after another on the single-root engine "
                            "(sum of tuples / sum of search times)",
        "mean_batch": round(float(np.mean([i["batch_size"] for i in infos])), 2),
        "batched_fraction": round(float(np.mean([i["batched"] for i in infos])), 3),
        "note": "at the offered rate the served rate is bounded by the arrivals (tuples of the "
                "requests per second); the saturated run gives the capacity",
    }
    if binfos:
        bspan = max(i["t_done"] for i in binfos) - min(i["t_submit"] for i in binfos)
        bm = sum(pool[gi]["m"][ri] for gi, ri in bpicks)
        bt = sum(pool[gi]["t_single"][ri] for gi, ri in bpicks)
        blat = np.array([i["t_done"] - i["t_submit"] for i in binfos]) * 1e3
        out["saturated"] = {
            "requests": len(binfos), "achieved_qps": round(len(binfos) / bspan, 1),
            "gteps": round(bm / bspan / 1e9, 4),
            "single_root_gteps_same_requests": round(bm / bt / 1e9, 4),
            "mean_batch": round(float(np.mean([i["batch_size"] for i in binfos])), 2),
            "batched_fraction": round(float(np.mean([i["batched"] for i in binfos])), 3),
            "latency_ms": {"p50": round(float(np.percentile(blat, 50)), 3),
                           "p99": round(float(np.percentile(blat, 99)), 3)},
        }
        log(f"[bench] serving saturated: {out['saturated']['achieved_qps']} qps, "
            f"{out['saturated']['gteps']} GTEPS (single-root alone "
            f"{out['saturated']['single_root_gteps_same_requests']}), mean batch "
            f"{out['saturated']['mean_batch']}, batched {out['saturated']['batched_fraction']}")
    log(f"[bench] serving: {out['achieved_qps']} qps, p50 {out['latency_ms']['p50']} ms, "
        f"p99 {out['latency_ms']['p99']} ms, {out['gteps']} GTEPS (single-root alone "
        f"{out['single_root_gteps_same_requests']}), mean batch {out['mean_batch']}, "
        f"batched {out['batched_fraction']}")
    del pool
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of the level loop is a design note, not a measured path", flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1208_5542_amd import csbfs, inputs

    wl = inputs.WORKLOADS[args.workload]
    n, p = wl.n, wl.p
    torch.cuda.set_device(0)
    t = time.perf_counter()
    src, dst = wl.tuples()
    log(f"[bench] generated {wl.name}: n={n} tuples={len(src)} in {time.perf_counter() - t:.1f}s")
    roots = wl.roots(src, dst, args.warmup + args.steps)
    if len(roots) < args.warmup + args.steps:
        raise SystemExit("not enough eligible roots")
    t = time.perf_counter()
    g = csbfs.Graph(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n, p)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"[bench] graph built p={p} nnz={g.info.nnz} max_block={g.info.max_block_nnz} "
        f"device={g.info.device_bytes / 2**30:.2f} GiB in {time.perf_counter() - t:.1f}s")
    flags = csbfs.FLAG_NO_SIEVE if args.no_sieve else 0
    flags |= {"auto": 0, "sparse": csbfs.FLAG_SPARSE_ONLY, "dense": csbfs.FLAG_DENSE_ONLY,
              "bottom_up": csbfs.FLAG_BOTTOM_UP_ONLY}[args.mode]
    # the timed pass runs uninstrumented (no per-kernel events, no counter
    # readback); a second pass over the same roots with per-kernel timing
    # gives the byte counts, the time split and the roofline
    eng = csbfs.Engine(g, max_levels=256, flags=flags)
    probe = csbfs.Engine(g, max_levels=256, flags=flags | csbfs.FLAG_TIMING)
    if args.alpha is not None or args.beta is not None:
        a_ = 16.0 if args.alpha is None else args.alpha
        b_ = 48.0 if args.beta is None else args.beta
        eng.set_direction(a_, b_)
        probe.set_direction(a_, b_)
    level = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    for r in roots[: args.warmup]:
        eng.bfs(int(r), level, parent, with_stats=False)
        probe.bfs(int(r), level, parent)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} roots)")

    stream = torch.cuda.current_stream()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    m_of = []
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k, r in enumerate(roots[args.warmup:]):
        ev0[k].record(stream)
        eng.bfs(int(r), level, parent, with_stats=False)
        ev1[k].record(stream)
        m_of.append(g.traversed_tuples(level))  # outside the recorded events
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    times = [ev0[k].elapsed_time(ev1[k]) / 1e3 for k in range(args.steps)]
    ms = [t * 1e3 for t in times]
    teps = [m / t for m, t in zip(m_of, times)]
    hmean = len(teps) / sum(1.0 / x for x in teps)
    log(f"[bench] timed {args.steps} roots in {wall:.2f}s wall; hmean {hmean / 1e9:.3f} GTEPS")
    per_root = []
    for r, m in zip(roots[args.warmup:], m_of):
        res = probe.bfs(int(r), level, parent)
        per_root.append((int(r), res.n_levels, res.stats, m, probe.stream_words(res.n_levels)))

    # bytes and compression over every message of every timed root
    tot = {k: 0 for k in ("raw_bytes", "wah_unsieved_bytes", "wah_sieved_bytes", "self_bytes",
                          "sieved_bits", "unsieved_bits", "edges", "view_bits")}
    inv_ratio, nlev = 0.0, 0
    # per kernel: algorithmic bytes (the formulas of expansion_bytes and
    # codec_bytes), event time, launches; the expansion also by direction
    kern = {k: [0, 0.0, 0] for k in ("expansion", "top_down", "top_down_binned", "bottom_up", "encode", "decode")}
    dir_count = {"top_down": 0, "bottom_up": 0, "top_down_binned": 0}
    # the search forms f^k inside the encoder of its messages: one category
    cat_ms = {"expand": 0.0, "update_compress": 0.0, "decode": 0.0}
    R = n // p
    for _, nl, stats, _m, _w in per_root:
        for k, s in enumerate(stats):
            for key in tot:
                tot[key] += s[key]
            if k > 0 and s["wah_sieved_bytes"] > 0:
                inv_ratio += s["wah_sieved_bytes"] / s["raw_bytes"]
                nlev += 1
            b = expansion_bytes(s, n, p)
            t = s["ms_expand"] + s["ms_long_rows"]
            d = "bottom_up" if s["direction"] == csbfs.DIR_BOTTOM_UP else "top_down"
            dir_count[d] += 1
            keys = ["expansion", d]
            if d == "top_down" and s["push"] == csbfs.PUSH_BINNED:
                dir_count["top_down_binned"] += 1
                keys.append("top_down_binned")  # a subset of top_down
            for key in keys:
                kern[key][0] += b
                kern[key][1] += t
                kern[key][2] += 1
            if k > 0:
                eb, db = codec_bytes(s, n, p)
                kern["encode"][0] += eb
                kern["encode"][1] += s["ms_compress"]
                kern["encode"][2] += 1
                kern["decode"][0] += db
                kern["decode"][1] += s["ms_decode"]
                kern["decode"][2] += 1
            cat_ms["expand"] += t
            cat_ms["update_compress"] += s["ms_update"] + s["ms_compress"]
            cat_ms["decode"] += s["ms_decode"]
    if p > 1:
        ratio = tot["raw_bytes"] / max(tot["wah_sieved_bytes"], 1)
        sieve_gain = tot["wah_unsieved_bytes"] / max(tot["wah_sieved_bytes"], 1)
        c_factor = inv_ratio / max(nlev, 1)
    else:  # one processor: only the self stream exists
        raw_self = sum((len(st) - 1) * 8 * (R // 64) for _, _, st, _, _ in per_root)
        ratio = raw_self / max(tot["self_bytes"], 1)
        sieve_gain = None
        c_factor = None
    # mode switch (Table 5: BIT / WAH / DIR-WAH) beside a Table-2 sparse vector,
    # per level summed over the timed roots: Alg. 1 sends every piece as a
    # raw bitmap, Alg. 2 its WAH stream, Alg. 3 the sieved WAH stream; a
    # sparse vector sends 8-byte ids of the piece to the p - 1 others
    by_level = {}
    for _, _nl, stats, _m, _w in per_root:
        for k, st_ in enumerate(stats):
            if k == 0:
                continue  # seeded, never sent
            d = by_level.setdefault(k, {"frontier": 0, "bit": 0, "wah": 0, "dir_wah": 0, "sparse": 0})
            d["frontier"] += st_["frontier"]
            d["bit"] += st_["raw_bytes"]
            d["wah"] += st_["wah_unsieved_bytes"]
            d["dir_wah"] += st_["wah_sieved_bytes"]
            d["sparse"] += 8 * (p - 1) * st_["frontier"]
    mode_levels, switch_total = [], 0
    for k in sorted(by_level):
        d = by_level[k]
        best = min(("bit", "wah", "dir_wah", "sparse"), key=lambda x: d[x])
        switch_total += d[best]
        mode_levels.append(dict(level=k, **d, cheapest=best))
    mode_switch = {
        "levels": mode_levels,
        "total": {x: sum(d[x] for d in by_level.values()) for x in ("bit", "wah", "dir_wah", "sparse")},
        "per_level_cheapest_total": switch_total,
        "note": "bytes sent between processors (i != j) over all timed roots; level 0 is seeded",
    } if p > 1 else None
    def rate(key):
        b, ms_, launches = kern[key]
        gbs = b / (ms_ / 1e3) / 1e9 if ms_ > 0 else 0.0
        return {"achieved": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 5),
                "algorithmic_bytes_per_launch": round(b / max(launches, 1)),
                "avg_launch_ms": round(ms_ / max(launches, 1), 5), "launches": launches}
    exp = rate("expansion")
    traffic = load_traffic(wl.name)
    # Sec. VI.A: the volume of each processor over a whole search (sent +
    # received WAH bytes, self streams left out), max over processors,
    # averaged over the timed roots
    vols = []
    for _, nl, _st, _m, words in per_root:
        w = words[1:nl].astype(np.int64)
        off = ~np.eye(p, dtype=bool)
        sent = (8 * w * off).sum(axis=(0, 2))
        recv = (8 * w * off).sum(axis=(0, 1))
        vols.append(int((sent + recv).max()) if p > 1 else 0)

    out = {
        "metric": METRIC,
        "value": round(hmean / 1e9, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sum(ms) / len(ms), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl.name, "graph": "R-MAT", "scale": wl.scale,
                   "edgefactor": wl.edgefactor, "initiator": [0.57, 0.19, 0.19, 0.05],
                   "n": n, "n_tuples": len(src), "p": p, "grid": f"{p}x{p}",
                   "roots": args.steps, "sieve": not args.no_sieve, "mode": args.mode},
        "compression_ratio": round(ratio, 3),
        "sieve_gain": None if sieve_gain is None else round(sieve_gain, 3),
        "paper_C_factor": None if c_factor is None else round(c_factor, 5),
        "bytes": {"raw": tot["raw_bytes"], "wah_unsieved": tot["wah_unsieved_bytes"],
                  "wah_sieved": tot["wah_sieved_bytes"], "self": tot["self_bytes"],
                  "bits_before_sieve": tot["unsieved_bits"], "bits_after_sieve": tot["sieved_bits"]},
        "time_split_ms": {k: round(v / args.steps, 4) for k, v in cat_ms.items()},
        "levels_by_direction": dir_count,
        "mode_switch": mode_switch,
        "volume_bytes": {"mean_over_roots": round(float(np.mean(vols)), 1), "max_over_roots": max(vols),
                         "note": "Sec. VI.A: max over processors of the WAH bytes a processor sends plus "
                                 "receives over one whole search"},
        "roofline": {"bound": "hbm",
                     "kernel": "expansion step of one level: level_kernel (top-down push or bottom-up pull, "
                               "chosen per level; level_kernel_wide on graphs of 2^24 vertices or more) + "
                               "expand_big_kernel (top-down long rows; on binned levels "
                               "their pairs go into bins) + bin_resolve_kernel (binned levels); time = the "
                               "kernels' own HIP-event intervals on the library's stream",
                     "achieved": exp["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": exp["frac"],
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": exp["algorithmic_bytes_per_launch"],
                     "avg_launch_ms": exp["avg_launch_ms"],
                     "by_direction": {"top_down": rate("top_down"), "bottom_up": rate("bottom_up"),
                                      "top_down_binned": rate("top_down_binned")},
                     "other_kernels": {"frontier_encode_kernel (update + sieve + compress)": rate("encode"),
                                       "search_decode_kernel (decode/merge + reduction)": rate("decode")}},
        "wall_s": round(wall, 3),
    }
    if not args.no_batched:
        del eng, probe, g, level, parent
        torch.cuda.empty_cache()
        out["batched"] = batched_section(args)
    if not args.no_serving:
        out["serving"] = serving_section(args)
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, host_cores())
        log(f"[bench] CPU oracle baseline on {workers} processes ...")
        out["cpu_baseline"] = cpu_baseline(n, src, dst, p, roots[args.warmup:], workers)
    if args.json_out:
        detail = dict(out)
        detail["per_root"] = [{"root": r, "levels": nl, "m": m, "ms": t, "stats": st}
                              for (r, nl, st, m, _w), t in zip(per_root, ms)]
        with open(args.json_out, "w") as f:
            json.dump(detail, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
