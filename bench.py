#!/usr/bin/env python3
"""Benchmark of the Frank-Wolfe hot path (LDS, Alg. 1) on one MI355X.

One step = one pass of the hot path over one synthetic graph whose edge
list is already resident in HBM: device ingest (canonical simple graph,
degree renumbering, CSR, sweep plan), N Frank-Wolfe iterations with the
exact duality gap, and the float view of the loads.  The metric is
edge-updates per second, m * N / step time.  The dominant kernel is the FW
sweep; its roofline line uses the sweep launches' HIP-event time and the
algorithmic bytes of one launch (8.25 B per edge-update: two 4-byte slot ids
and two decision bits; 16 B per row: own key read and new key written).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lds_large]
Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Hardware queues per process for the HIP runtime (its default is 4): the
# serving section runs a scheduler, four batch streams and twelve worker
# streams at once, whose small kernels otherwise wait behind each other on
# four queues (20 s at 200 QPS offered: 137 completions/s with 4, 160 with 8,
# 172 with 16).  Read by the runtime when it starts, so it is set before
# torch or the library touch the GPU (LDS_BENCH_HW_QUEUES chooses another
# count, at most 32).  The single-stream sections do not depend on it.
HW_QUEUES = str(min(32, max(1, int(os.environ.get("LDS_BENCH_HW_QUEUES", "16")))))
os.environ["GPU_MAX_HW_QUEUES"] = HW_QUEUES

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    """the host CPU's model name (from /proc/cpuinfo), or 'unknown'"""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2504_10937_amd", "csrc", "fw.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per sweep launch from the committed rocprofv3 PMC summary, if
    it was taken on the current sweep kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "fw_sweep_%s_pmc.md" % workload)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = re.search(r"kernel source sha256\[:16\]:\s*`?([0-9a-f]{16})", txt)
    b = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", txt)
    if not h or not b or h.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def bench_batched(lds, torch, synth, np, count, plain=True):
    """The uneven-batch workload: graph g = batch member g (seed 1000 + g),
    even g edge density with 100 FW iterations, odd g triangle density with
    200.  Batched: one run of the captured persistent launch (tuned launch
    shape); plain: lds_frank_wolfe graph by graph.  Both start from the
    canonical initial point; the loads must agree bit for bit."""
    log("batched: %d graphs" % count)
    ms = []
    for i in range(count):
        n, s, d = synth.batch_member(i)
        mode = 2 if i % 2 == 0 else 3
        ms.append((n, s, d, mode, 100 if mode == 2 else 200))
    gs = [lds.lds_create_graph(n, s, d) for n, s, d, _, _ in ms]
    modes = [m[3] for m in ms]
    iters = [m[4] for m in ms]
    cache = os.path.join(ROOT, "paper_2504_10937_amd", "tune_cache.json")
    tune, tuned_ms = lds.lds_batch_autotune(gs, modes, iters, cache_path=cache, reps=1)
    log("batched: tune %s (%s)" % (tune.as_dict(), "cached" if tuned_ms < 0 else "timed"))
    b = lds.lds_batch_create(gs, modes, iters, tune=tune)
    lds.lds_batch_run(b)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        lds.lds_batch_run(b)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    info = lds.lds_batch_info(b, want_ms=True)
    tp, same = float("nan"), None
    if plain:
        nums = [lds.lds_loads(g, m, want_num=True)["num"] for g, m in zip(gs, modes)]
        t0 = time.perf_counter()
        for g, m, it in zip(gs, modes, iters):
            lds.lds_frank_wolfe(g, m, it)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        same = all(np.array_equal(lds.lds_loads(g, m, want_num=True)["num"], a) for g, m, a in zip(gs, modes, nums))
    work = sum((lds.lds_sweep_info(g, m)["slots"]) * it for g, m, it in zip(gs, modes, iters))
    del b
    # the same comparison with the FP64 gap of every iteration on both sides
    # (LDS_BATCH_GAP; lds_frank_wolfe with the gap): loads bit for bit and
    # gaps within FP64 rounding of the same exact sums
    bg = lds.lds_batch_create(gs, modes, iters, gap=True, tune=tune)
    lds.lds_batch_run(bg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lds.lds_batch_run(bg)
    torch.cuda.synchronize()
    tbg = (time.perf_counter() - t0) / reps
    gap_res = {"batched_ms": tbg * 1e3, "batched_graphs_per_s": count / tbg}
    if plain:
        states = [lds.lds_loads(g, m, want_num=True, want_gap=True) for g, m in zip(gs, modes)]
        t0 = time.perf_counter()
        for g, m, it in zip(gs, modes, iters):
            lds.lds_frank_wolfe(g, m, it, want_gap=True)
        torch.cuda.synchronize()
        tpg = time.perf_counter() - t0
        same_g = True
        for g, m, st in zip(gs, modes, states):
            now = lds.lds_loads(g, m, want_num=True, want_gap=True)
            same_g = same_g and np.array_equal(now["num"], st["num"]) and \
                bool(np.allclose(now["gap"], st["gap"], rtol=1e-12, atol=0.0))
        gap_res.update({"plain_ms": tpg * 1e3, "plain_graphs_per_s": count / tpg, "speedup": tpg / tbg,
                        "identical": same_g})
    del bg
    for g in gs:
        g.destroy()
    res = {"graphs": count, "batched_graphs_per_s": count / tb, "plain_graphs_per_s": count / tp,
           "speedup": tp / tb, "batched_ms": tb * 1e3, "plain_ms": tp * 1e3, "kernel_ms": info["kernel_ms"],
           "kernel_graphs": info["kernel_graphs"], "plain_path_graphs": info["plain_graphs"],
           "incidence_updates_per_s": work / tb, "bit_identical": same, "tune": info["tune"],
           "with_fp64_gap": gap_res}
    log("batched: %.1f ms vs plain %.1f ms (x%.1f), identical %s; with the gap %.1f ms vs %s ms" %
        (tb * 1e3, tp * 1e3, tp / tb, same, tbg * 1e3, "%.1f" % gap_res["plain_ms"] if plain else "-"))
    return res


def bench_density(lds, torch, synth, densities):
    """The scalability experiment's density sweep: Barabasi-Albert graphs with
    n = 1M and density d (m = d n); LDScvx (lds_topk, k = 5, N = 100) end to
    end from the resident edge list, and the FW sweep rate alone."""
    res = {}
    for d in densities:
        n, s, t, mode, iters, k = synth.workload("ba_d%d" % d)
        ts, tt = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = lds.lds_create_graph(n, ts, tt)
        sets, st = lds.lds_topk(g, mode, k, iters, with_stats=True)
        t1 = time.perf_counter()
        fw_ms, launches = 0.0, 0
        lds.lds_frank_wolfe(g, mode, iters)
        fw_ms, launches = lds.lds_fw_elapsed(g, mode)
        m = lds.lds_graph_info(g)["m"]
        res["ba_d%d" % d] = {"n": n, "m": m, "ldscvx_s": t1 - t0, "lds_found": len(sets),
                             "top_density": str(sets[0][1]) if sets else None,
                             "fw_edge_updates_per_s": m * iters / (fw_ms / 1e3),
                             "phases_ms": {x: round(st[x], 1) for x in ("ms_core", "ms_fw", "ms_prune", "ms_search")}}
        log("density %d: LDScvx %.2f s, FW %.2f ms" % (d, t1 - t0, fw_ms))
        g.destroy()
    return res


def bench_topk(lds, torch, synth, names):
    """LDScvx / LTDScvx end to end (lds_topk with the workload's k and N) from
    the resident edge list of the large edge workload and the LTDS workload."""
    res = {}
    for name in names:
        n, s, t, mode, iters, k = synth.workload(name)
        ts, tt = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = lds.lds_create_graph(n, ts, tt)
        sets, st = lds.lds_topk(g, mode, k, iters, with_stats=True)
        t1 = time.perf_counter()
        g.destroy()
        res[name] = {"k": k, "fw_iters": iters, "mode": "edge" if mode == 2 else "triangle", "seconds": t1 - t0,
                     "found": len(sets), "top_density": str(sets[0][1]) if sets else None,
                     "stats": {x: (round(v, 1) if isinstance(v, float) else v) for x, v in st.items()}}
        log("topk %s: %.2f s, %d sets" % (name, t1 - t0, len(sets)))
    return res


def bench_ltds(lds, torch, synth, name):
    """The triangle program (Eq. trcp, Alg. 6) on the LTDS workload: device
    triangle listing, N exact FW iterations with the gap, sort / prefix /
    stable groups; sweep rate against the HBM roofline (2 payload ids, one
    decision bit per slot, 16 B per row)."""
    n, s, t, mode, iters, _ = synth.workload(name)
    ts, tt = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
    g = lds.lds_create_graph(n, ts, tt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = lds.lds_triangles(g)[0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lds.lds_frank_wolfe(g, mode, iters, want_gap=True)
    t2 = time.perf_counter()
    groups, _, _ = lds.lds_stable_groups(g, mode)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    fw_ms, launches = lds.lds_fw_elapsed(g, mode)
    sw = lds.lds_sweep_info(g, mode)
    per_launch_s = fw_ms / 1e3 / max(launches, 1)
    alg = sw["slots"] * 8 + sw["slots"] / 8.0 + sw["rows"] * 16.0
    achieved = alg / per_launch_s / 1e9
    g.destroy()
    log("ltds %s: T=%d listing %.1f ms, FW %.1f ms, groups %.1f ms" % (name, T, (t1 - t0) * 1e3, fw_ms,
                                                                   (t3 - t2) * 1e3))
    return {"workload": name, "n": n, "triangles": T, "fw_iters": iters, "triangle_listing_ms": (t1 - t0) * 1e3,
            "fw_wall_ms": (t2 - t1) * 1e3, "fw_sweep_ms": fw_ms, "sort_prefix_groups_ms": (t3 - t2) * 1e3,
            "groups": len(groups), "triangle_updates_per_s": T * iters / (fw_ms / 1e3),
            "sweep_ms_per_launch": per_launch_s * 1e3,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name),
                         "alg_bytes_per_launch": alg, "kernel": "k_fw_sweep<3>"}}


def bench_clique4(lds, torch, synth, name):
    """The 4-clique program (h = 4): device listing of the 4-cliques from the
    triangles, then N exact FW iterations with the gap; sweep rate against the
    HBM roofline with the same per-slot byte count as the edge and triangle
    sweeps (h-1 payload ids, one decision bit, 16 B per row)."""
    n, s, t, mode, iters, _ = synth.workload(name)
    ts, tt = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
    g = lds.lds_create_graph(n, ts, tt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lds.lds_triangles(g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Q = lds.lds_cliques4(g)[0]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lds.lds_frank_wolfe(g, mode, iters, want_gap=True)
    t3 = time.perf_counter()
    fw_ms, launches = lds.lds_fw_elapsed(g, mode)
    sw = lds.lds_sweep_info(g, mode)
    per_launch_s = fw_ms / 1e3 / max(launches, 1)
    alg = sw["slots"] * 12 + sw["slots"] / 8.0 + sw["rows"] * 16.0
    achieved = alg / per_launch_s / 1e9
    g.destroy()
    log("clique4 %s: Q=%d listing %.1f ms, FW %.1f ms" % (name, Q, (t2 - t1) * 1e3, fw_ms))
    return {"workload": name, "n": n, "cliques4": Q, "fw_iters": iters,
            "triangle_listing_ms": (t1 - t0) * 1e3, "clique_listing_ms": (t2 - t1) * 1e3,
            "fw_wall_ms": (t3 - t2) * 1e3, "fw_sweep_ms": fw_ms,
            "clique_updates_per_s": Q * iters / (fw_ms / 1e3),
            "sweep_ms_per_launch": per_launch_s * 1e3,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name),
                         "alg_bytes_per_launch": alg, "kernel": "k_fw_sweep<4>"}}


def _serve_run(lds, np, srv, gs, seconds, qps, seed, tag0, keep=0):
    """Offer a Poisson stream of `qps` queries per second for `seconds`; wait
    for all of them.  keep: return the result sets of the first `keep`
    queries (by position in the stream) for the identity check."""
    import synth
    q = synth.queries(int(seconds * qps * 1.5) + 16, qps=qps, pool=len(gs), kmax=10, seed=seed)
    ta = q["t_arrive"]
    n = int((ta < seconds).sum())
    base = lds.lds_server_clock(srv)
    done = []
    i = 0
    while len(done) < n:
        now = lds.lds_server_clock(srv) - base
        while i < n and ta[i] <= now:
            mode = int(q["mode"][i])
            lds.lds_server_submit(srv, gs[int(q["graph"][i])], mode, int(q["k"][i]), 100 if mode == 2 else 200,
                                  tag0 + i, base + float(ta[i]))
            i += 1
        wait = min(0.05, max(0.0, float(ta[i]) - now)) if i < n else 0.2
        done.extend(lds.lds_server_poll(srv, 256, wait))
    lat = np.array([c["t_done"] - c["t_arrive"] for c in done])
    span = max(c["t_done"] for c in done) - base
    errs = sum(c["status"] != 0 for c in done)
    in_window = sum(c["t_done"] - base <= seconds for c in done)
    # completed_per_s: all queries over the time to the last completion (the
    # drain of the last ones included); completed_in_window_per_s: what the
    # server finished while queries were arriving, against arrived_per_s
    res = {"offered_qps": qps, "arrival_window_s": seconds, "queries": n, "errors": errs,
           "completed_per_s": n / span, "arrived_per_s": n / seconds,
           "completed_in_window_per_s": in_window / seconds, "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3)}
    kept = {c["tag"] - tag0: c["sets"] for c in done if c["tag"] - tag0 < keep}
    return res, q, kept


def bench_serving(lds, torch, synth, np, seconds, qps, ladder, plain_sample, p99_bound_ms=2000.0, workers=12,
                  ladder_seconds=12.0):
    """The serving workload: a resident pool of 64 graphs (pool member g,
    seed 5 + g, graph 0 pinned at n = 2M), Poisson arrivals, graph uniform
    over the pool, LDS / LTDS half and half (100 / 200 FW iterations), k
    uniform in 1..10.  Latency = completion - arrival on the server clock.
    Reported: the offered load for `seconds` after a warm-up; the highest
    offered rate of the ladder at which the server keeps up (its completions
    during the arrival window reach 95% of the arrivals) with p99 within the
    bound; and the plain baseline: the
    first `plain_sample` queries of the offered stream through lds_topk one
    at a time on the same resident graphs, with their results compared to the
    served ones."""
    log("serving: building the pool")
    pool = [synth.pool_member(i) for i in range(64)]
    gs = [lds.lds_create_graph(*p) for p in pool]
    for g in gs:
        lds.lds_triangles(g)
    torch.cuda.synchronize()
    srv = lds.lds_server_create(0, max_slots=64, workers=workers)
    # warm-up: one query per (graph, mode), so that each graph's resident
    # host data (adjacency, core numbers) exists
    for i, g in enumerate(gs):
        for m in (2, 3):
            lds.lds_server_submit(srv, g, m, 3, 100 if m == 2 else 200, 10 ** 9 + 2 * i + m)
    got = 0
    while got < 2 * len(gs):
        got += len(lds.lds_server_poll(srv, 256, 1.0))
    res = {"pool_graphs": len(gs), "pool_vertices": int(sum(p[0] for p in pool)),
           "pool_edges": int(sum(len(p[1]) for p in pool)), "workers": workers, "hw_queues": int(HW_QUEUES)}
    log("serving: %g QPS for %g s" % (qps, seconds))
    res["offered"], stream, served = _serve_run(lds, np, srv, gs, seconds, qps, 5, 0, keep=plain_sample)
    log("serving: %s" % res["offered"])
    steps = []
    for k, rate in enumerate(ladder):
        r, _, _ = _serve_run(lds, np, srv, gs, ladder_seconds, rate, 60 + k, 10 ** 6 * (k + 1))
        steps.append(r)
        log("serving ladder: %s" % r)
    res["ladder"] = steps
    ok = [r["offered_qps"] for r in steps
          if r["completed_in_window_per_s"] >= 0.95 * r["arrived_per_s"] and r["p99_ms"] <= p99_bound_ms
          and r["errors"] == 0]
    res["max_sustained_qps"] = max(ok) if ok else None
    res["sustain_rule"] = ("completions during the arrival window >= 95%% of the arrivals and p99 <= %g ms, "
                           "over a %g s arrival window" % (p99_bound_ms, ladder_seconds))
    st = lds.lds_server_stats(srv)
    res["batches"] = st["batches"]
    res["max_batch"] = st["max_batch"]
    res["peak_inflight_bytes"] = st["peak_inflight_bytes"]
    lds.lds_server_destroy(srv)
    if plain_sample > 0:
        m = min(plain_sample, res["offered"]["queries"])
        same = True
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(m):
            mode = int(stream["mode"][i])
            sets = lds.lds_topk(gs[int(stream["graph"][i])], mode, int(stream["k"][i]), 100 if mode == 2 else 200)
            mine = served.get(i)
            same = same and mine is not None and len(mine) == len(sets) and all(
                a[1] == b[1] and np.array_equal(a[0], b[0]) for a, b in zip(mine, sets))
        tp = time.perf_counter() - t0
        res["plain"] = {"queries": m, "queries_per_s": m / tp, "identical_to_served": bool(same),
                        "how": "the offered stream's first queries, lds_topk one at a time on the resident graphs"}
        res["served_vs_plain"] = res["offered"]["completed_per_s"] / (m / tp)
        log("serving plain: %d queries at %.1f/s, identical %s" % (m, m / tp, same))
    for g in gs:
        g.destroy()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lds_large")
    ap.add_argument("--cpu-iters", type=int, default=4, help="FW iterations of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fw-only", action="store_true", help="leave the sort / prefix / stable groups out of the step")
    ap.add_argument("--iters", type=int, default=0, help="override the workload's FW iteration count")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (a known-size kernel for counter scaling)")
    ap.add_argument("--batch-graphs", type=int, default=4096,
                    help="graphs of the batched-vs-plain comparison (0: skip)")
    ap.add_argument("--no-batch-plain", action="store_true",
                    help="leave out the per-graph comparison of the batched section (shorter kernel traces)")
    ap.add_argument("--density-sweep", default="2,4,6,8,10,12",
                    help="Barabasi-Albert densities of the scalability section (n = 1M; empty: skip)")
    ap.add_argument("--copy-gib", type=float, default=1.0,
                    help="GiB copied by the library's streaming copy kernel for the bandwidth ceiling (0: skip)")
    ap.add_argument("--cpu-reps", type=int, default=3, help="timed repetitions of the oracle sample (median)")
    ap.add_argument("--ltds", default="ltds_hk", help="triangle (LTDS) workload ('' to skip)")
    ap.add_argument("--topk", default="lds_large,ltds_hk", help="workloads timed end to end by lds_topk ('' to skip)")
    ap.add_argument("--clique4", default="clique4_pl", help="4-clique FW workload ('' to skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="arrival window of the serving run (0: skip)")
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-ladder", default="50,100,150,175,190",
                    help="offered rates (QPS) tried for the highest sustained load ('' to skip)")
    ap.add_argument("--serve-workers", type=int, default=12, help="verification worker threads of the server")
    ap.add_argument("--serve-ladder-seconds", type=float, default=12.0, help="arrival window of each ladder rate")
    ap.add_argument("--serve-plain", type=int, default=200,
                    help="queries of the offered stream also run one at a time by lds_topk (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (one process, one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2504_10937_amd as lds

    assert torch.cuda.is_available(), "no HIP device"
    lds.load()
    lds.lds_set_allocator(True)  # library buffers from torch's caching allocator
    if args.copy_calib_mib:
        x = torch.empty(args.copy_calib_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    n, src, dst, mode, iters, k = synth.workload(args.workload)
    if args.iters:
        iters = args.iters
    log("workload %s: n=%d pairs=%d mode=%d N=%d" % (args.workload, n, len(src), mode, iters))
    ts = torch.from_numpy(src).cuda()
    td = torch.from_numpy(dst).cuda()
    r = torch.empty(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    phases = {}

    def step():
        t = [time.perf_counter()]
        g = lds.lds_create_graph(n, ts, td, stream=stream)
        if mode == 3:
            lds.lds_triangles(g, stream=stream)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        lds.lds_frank_wolfe(g, mode, iters, r_out=r, want_gap=True, stream=stream)
        t.append(time.perf_counter())
        groups = None
        if not args.fw_only:
            groups, _, _ = lds.lds_stable_groups(g, mode, stream=stream)
        t.append(time.perf_counter())
        fw_ms, launches = lds.lds_fw_elapsed(g, mode)
        info = lds.lds_graph_info(g)
        sw = lds.lds_sweep_info(g, mode, stream=stream)
        g.destroy()
        for k, (a, b) in zip(("ingest", "fw", "sort_prefix_groups"), zip(t, t[1:])):
            phases.setdefault(k, []).append((b - a) * 1e3)
        phases.setdefault("groups", []).append(len(groups) if groups is not None else -1)
        return fw_ms, launches, info, sw

    for i in range(args.warmup):
        step()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    fw_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ms, launches, info, sw = step()
        fw_ms.append(ms)
        log("step %d: sweep launches %.3f ms" % (i, ms))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    m = info["m"]
    units = m if mode == 2 else info["triangles"]
    value = units * iters / (ms_step / 1e3)
    fw_mean = sum(fw_ms) / len(fw_ms)
    per_launch_s = fw_mean / 1e3 / max(launches, 1)
    slot_bytes = 4 * (mode - 1)
    alg_bytes = sw["slots"] * slot_bytes + sw["slots"] / 8.0 + sw["rows"] * 16.0
    achieved = alg_bytes / per_launch_s / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": "FW edge-updates/s" if mode == 2 else "FW triangle-updates/s",
        "value": value,
        "unit": "edge-updates/s" if mode == 2 else "triangle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "triangles": info["triangles"], "fw_iters": iters,
                   "mode": "edge" if mode == 2 else "triangle", "step": "ingest+fw(gap)+float view" + ("" if args.fw_only else "+sort/prefix/stable groups")},
        "fw_only_updates_per_s": units * iters / (fw_mean / 1e3),
        "phase_ms": {k: sum(v) / len(v) for k, v in phases.items()},
        "fw_sweep_ms_per_launch": per_launch_s * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "kernel": "k_fw_sweep"},
    }
    if args.copy_gib > 0:
        nb = int(args.copy_gib * (1 << 30)) // 16 * 16
        x = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        cms = lds.lds_copy_bandwidth(y, x, reps=10)
        del x, y
        copy_gbs = 2.0 * nb / (cms / 1e3) / 1e9
        out["roofline"]["copy_ceiling"] = {"achieved": copy_gbs, "unit": "GB/s", "kernel": "k_copy16",
                                           "bytes_per_copy": 2 * nb, "ms_per_copy": cms}
        out["roofline"]["frac_of_copy"] = achieved / copy_gbs
        log("copy ceiling: %.0f GB/s (%.3f ms per %.2f GiB copy)" % (copy_gbs, cms, args.copy_gib))
        # the random-gather ceiling over a table of n codes (the sweep gathers
        # the 16-bit code of every neighbour outside its LDS cache)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        ng = 1 << 26
        idx = torch.randint(0, n, (ng,), dtype=torch.int32, device="cuda", generator=gen)
        table = torch.zeros(n, dtype=torch.int16, device="cuda")
        gms = lds.lds_gather_rate(idx, table, reps=5)
        del idx, table
        out["roofline"]["gather_ceiling"] = {"gathers_per_s": ng / (gms / 1e3), "table_bytes": 2 * n,
                                             "kernel": "k_gather16", "indices": ng}
        log("gather ceiling: %.3g gathers/s over a %d-entry table" % (ng / (gms / 1e3), n))
    if args.batch_graphs > 0:
        out["batched"] = bench_batched(lds, torch, synth, np, args.batch_graphs, not args.no_batch_plain)
    if args.density_sweep:
        out["density_sweep"] = bench_density(lds, torch, synth, [int(x) for x in args.density_sweep.split(",")])
    if args.ltds:
        out["ltds"] = bench_ltds(lds, torch, synth, args.ltds)
    if args.topk:
        out["topk"] = bench_topk(lds, torch, synth, args.topk.split(","))
    if args.clique4:
        out["clique4"] = bench_clique4(lds, torch, synth, args.clique4)
    if args.serve_seconds > 0:
        out["serving"] = bench_serving(lds, torch, synth, np, args.serve_seconds, args.serve_qps,
                                       [float(x) for x in args.serve_ladder.split(",") if x], args.serve_plain,
                                       workers=args.serve_workers, ladder_seconds=args.serve_ladder_seconds)
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline: oracle ingest (untimed)")
        G = oracle.Graph(n, src, dst)
        times = []
        for _ in range(max(1, args.cpu_reps)):
            t = time.perf_counter()
            oracle.fw_exact(G, mode, args.cpu_iters, with_gap=True, with_split=False)
            times.append(time.perf_counter() - t)
        dt = sorted(times)[len(times) // 2]
        cpu_units = G.m if mode == 2 else oracle.num_patterns(G, mode)
        out["cpu_baseline"] = {
            "value": cpu_units * args.cpu_iters / dt, "unit": out["unit"], "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "sample": "%s graph (n=%d, m=%d), %d of the %d FW iterations incl. exact gap, single thread, "
                      "median of %d runs (%s s)" % (args.workload, n, G.m, args.cpu_iters, iters, len(times),
                                                   ", ".join("%.1f" % x for x in times))}
        log("cpu baseline: %.3g %s" % (out["cpu_baseline"]["value"], out["unit"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
