"""Benchmark: FORA whole-graph SSPPR + top-500 on one MI355X.

Workload (default, ``rmat23``): R-MAT, 2^23 nodes, 16 * 2^23 samples with
(a, b, c) = (.57, .19, .19), duplicates and self-loops removed, dangling
nodes given one random out-edge (about 136M edges, CSR int32); 1,024 seeded
sources drawn in proportion to out-degree (duplicates kept); alpha = 0.2,
eps = 0.5, delta = p_f = 1/n, k = 500.

Per-query state is dense, so the 1,024 sources run in four waves of 256
queries, each wave one batched call. One step = one wave: the whole hot path
(push, walk plan, walks, estimate, top-k) for 256 sources; successive steps
cycle through the four waves, so every four steps cover all 1,024 sources.
The plain single-query loop over a stated sample of the same sources is
timed beside it, and the CPU oracle on a stated bounded sample. Prints one
JSON line.

``--workload rmat20`` gives the single-query configuration instead (R-MAT
2^20, 100 sources uniform over nodes with R-MAT out-degree >= 1, one wave).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walk-steps/s + SSPPR queries/s (eps=0.5, top-500) vs plain FORA, same GPU"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes of the method on a CSR graph: per walk move 12 B (the
# row's two offsets and the chosen column index); per walk 8 B plan read
# (amortised) + 8 B fixed-point weight at the end point. The bench asks for
# no per-node walk counts, so no count update is charged.
BYTES_PER_STEP = 12
BYTES_PER_WALK = 16
# queries per batched call by workload (dense per-query state: about 52 bytes
# per node and query, so 256 queries of 2^23 nodes take ~112 GB of HBM)
DEFAULT_WAVE = {"rmat23": 256}
# launch shapes the library's autotuner chose on MI355X for these workloads
TUNING_CACHE = os.path.join(ROOT, "paper_1908_10583_amd", "tuning_mi355x.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_digest(paths) -> str:
    """SHA-256 of the sources' code (paths relative to the repository):
    comments removed and whitespace runs collapsed, so that a comment edit
    keeps a counter record valid and any change to the code does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for src in paths:
        text = open(os.path.join(ROOT, src)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
        h.update(b"\0")
    return h.hexdigest()


def recorded_traffic(kernel: str, tag: str):
    """HBM-side bytes per launch from the committed counter record for this
    workload (tag: workload and batch, e.g. rmat23_b256), or None if there is
    none or the kernel's code changed since the counters were taken."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_{tag}_traffic.json")):
        rec = json.load(open(path))
        try:
            digest = code_digest(rec["sources"])
        except OSError:
            continue
        if digest == rec.get("code_sha256"):
            return rec["traffic_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def _oracle_sample(args):
    """One bounded oracle query: the full push and walk plan, then the walks
    of the plan's first entries up to ``walk_budget`` walks. Returns the
    times and counts (run in a worker process)."""
    g, src, alpha, eps, seed, walk_budget = args
    import oracle
    n = g.n
    c = oracle.constants(g.m, alpha, eps, 1.0 / n, 1.0 / n)
    t0 = time.perf_counter()
    p = oracle.push(g, int(src), alpha, c["rmax"])
    t1 = time.perf_counter()
    pv, po, pw = oracle.plan(p["r"], c["omega_unit"])
    t2 = time.perf_counter()
    cum = np.cumsum(po.astype(np.int64))
    take = int(np.searchsorted(cum, walk_budget, side="right"))
    take = max(1, min(take, len(pv)))
    w = oracle.walks(g, int(src), seed, c["t_alpha"], pv[:take], po[:take], pw[:take])
    t3 = time.perf_counter()
    return dict(src=int(src), push_s=t1 - t0, plan_s=t2 - t1, walk_s=t3 - t2,
                walks_run=int(cum[take - 1]), walks_total=int(cum[-1]) if len(cum) else 0,
                steps=int(w["steps"]), edge_ops=int(p["edge_ops"]))


def cpu_baseline(g, srcs, alpha, eps, seed, walk_budget=3_000_000):
    """The CPU oracle (plain single-threaded FP64 C) on a bounded sample of
    the workload: per source the full push and plan, and the walks of the
    plan's first entries up to ``walk_budget`` walks; the rest of the query
    is extrapolated at the measured per-walk time. Run once on one core and
    then as one independent query per host core at once (fork)."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores or 1), 16))
    one = _oracle_sample((g, srcs[0], alpha, eps, seed, walk_budget))

    def per_query_s(r):
        per_walk = r["walk_s"] / max(r["walks_run"], 1)
        return r["push_s"] + r["plan_s"] + per_walk * r["walks_total"]

    q1 = per_query_s(one)
    multi = None
    if cores > 1:
        ctx = mp.get_context("fork")
        jobs = [(g, srcs[i % len(srcs)], alpha, eps, seed, walk_budget) for i in range(cores)]
        t0 = time.perf_counter()
        with ctx.Pool(cores) as pool:
            res = pool.map(_oracle_sample, jobs)
        wall = time.perf_counter() - t0
        steps = sum(r["steps"] for r in res)
        walk_wall = max(r["walk_s"] for r in res)
        multi = dict(cores=cores, wall_s=round(wall, 2),
                     walk_steps_per_s=steps / walk_wall,
                     queries_per_s_extrapolated=round(
                         cores / float(np.mean([per_query_s(r) for r in res])), 4))
    return dict(value=one["steps"] / one["walk_s"], unit="walk-steps/s", cores=1, kind="oracle",
                queries_per_s_extrapolated=round(1.0 / q1, 5),
                push_s=round(one["push_s"], 3), walk_s=round(one["walk_s"], 3),
                host_cores=cores, all_cores=multi,
                sample=(f"source {one['src']} (the workload's first): full push "
                        f"({one['edge_ops']} residue increments) and walk plan, then the first "
                        f"{one['walks_run']} of its {one['walks_total']} walks "
                        f"({one['steps']} walk steps); queries/s extrapolates the remaining "
                        f"walks at the measured per-walk time; all_cores runs one such query "
                        f"per host core at once"))


def small_graph_leg(alpha, eps, k, seed, cache, args, log):
    """One query at a time on R-MAT 2^20 (16.6M edges, 100 sources uniform
    over nodes with out-degree >= 1): queries/s and latency in the launch
    shape tuned for one query, then per-phase latency from the eager path's
    events. The graph fits in the 256 MB Infinity Cache, so this leg makes
    no HBM-roofline claim."""
    import torch
    import synth
    from paper_1908_10583_amd import autotune, fora

    g2, srcs2 = synth.workload("rmat20")
    G2 = fora.Graph.from_numpy(g2.rowptr, g2.colidx, device="cuda:0")
    tun = None
    if not args.no_autotune:
        one = fora.make_queries(srcs2[:1], alpha=alpha, eps=eps, k=k, seed=seed, n=g2.n)
        tun = dict(autotune.autotune(G2, one, path=cache, force=args.retune)["tuning"])
    ws1 = fora.workspace(G2, 1)
    o1 = (torch.empty(k, dtype=torch.int32, device="cuda:0"),
          torch.empty(k, dtype=torch.float32, device="cuda:0"))
    for s in srcs2[:2]:
        fora.fora_ssppr(G2, int(s), alpha, eps, k=k, seed=seed, ws=ws1, out=o1)
    torch.cuda.synchronize()
    lat, steps = [], 0
    t1 = time.perf_counter()
    for s in srcs2:
        ts = time.perf_counter()
        r = fora.fora_ssppr(G2, int(s), alpha, eps, k=k, seed=seed, ws=ws1, out=o1, stats=True)
        lat.append(time.perf_counter() - ts)
        steps += r.stats["steps"]
    dt = time.perf_counter() - t1
    G2.set_tuning(graph_rounds=0)
    ph = dict(ms_push=0.0, ms_plan=0.0, ms_walk=0.0, ms_topk=0.0)
    for s in srcs2:
        r = fora.fora_ssppr(G2, int(s), alpha, eps, k=k, seed=seed, ws=ws1, out=o1, stats=True)
        for key in ph:
            ph[key] += r.stats[key] / len(srcs2)
    out = dict(workload=f"{g2.name}: n={g2.n} m={g2.m}, {len(srcs2)} sources one at a time",
               queries_per_s=round(len(srcs2) / dt, 2), walk_steps_per_s=steps / dt,
               latency_ms_p50=round(float(np.median(lat)) * 1e3, 3),
               latency_ms_p99=round(float(np.percentile(lat, 99)) * 1e3, 3),
               eager_phases_ms={key: round(v, 3) for key, v in ph.items()}, tuning=tun)
    log(f"single queries on R-MAT 2^20: {out['queries_per_s']} q/s, p50 "
        f"{out['latency_ms_p50']} ms")
    G2.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat23")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even if the committed tuning cache has this workload")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--max-batch", type=int, default=None,
                    help="queries per batched call (0: all sources in one call)")
    ap.add_argument("--single-sample", type=int, default=None,
                    help="sources timed by the plain single-query loop (0: all)")
    ap.add_argument("--sources", type=int, default=0,
                    help="use only the workload's first N sources (0: all)")
    ap.add_argument("--leg-steps", type=int, default=None,
                    help="timed steps of each extra leg (default: 2 with waves, else --steps)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--no-alg3", action="store_true", help="skip the Algorithm 3 leg")
    ap.add_argument("--no-topk", action="store_true", help="skip the top-k FORA leg")
    ap.add_argument("--no-pagerank", action="store_true", help="skip the global PageRank leg")
    ap.add_argument("--no-index", action="store_true", help="skip the FORA+ (index) leg")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the single-query leg on R-MAT 2^20 (100 sources)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy, whose HBM counter "
                         "readings calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "a single-GPU benchmark: --gpus must be 1 (queries shard "
                                   "across GPUs by source, with no collective on the hot path)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1908_10583_amd import autotune, fora

    alpha, eps, k, seed = 0.2, 0.5, 500, 0
    t0 = time.perf_counter()
    g, srcs = synth.workload(args.workload)
    if args.sources:
        srcs = srcs[:args.sources]
    log(f"graph {g.name}: n={g.n} m={g.m} sources={len(srcs)} ({time.perf_counter()-t0:.1f}s)")
    G = fora.Graph.from_numpy(g.rowptr, g.colidx, device="cuda:0")
    B = len(srcs)
    max_batch = args.max_batch if args.max_batch is not None else \
        DEFAULT_WAVE.get(args.workload, 0)
    WB = min(B, max_batch) if max_batch else B
    waves = [(a, min(a + WB, B)) for a in range(0, B, WB)]
    qs_w = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n)
            for a, b in waves]
    multi = len(waves) > 1
    leg_steps = args.leg_steps if args.leg_steps is not None else (2 if multi else args.steps)
    leg_warmup = min(args.warmup, 1) if multi else args.warmup
    single_sample = args.single_sample if args.single_sample is not None else \
        (64 if multi else 0)
    ws_bytes = fora.fora_workspace_size(G, WB)
    if not args.no_topk:  # the top-k leg reuses it (staging rows after the main layout)
        ws_bytes = max(ws_bytes, fora.fora_topk_workspace_size(G, WB, k))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    ids = torch.empty((B, k), dtype=torch.int32, device="cuda:0")
    vals = torch.empty((B, k), dtype=torch.float32, device="cuda:0")
    log(f"workspace {ws.numel()/2**30:.2f} GiB for waves of {WB} ({len(waves)} waves)")

    def run_wave(i, stats=False, queries=None):
        a, b = waves[i]
        q = qs_w[i] if queries is None else queries[i]
        res = fora.fora_ssppr_batch(G, q, kmax=k, ws=ws, out=(ids[a:b], vals[a:b]),
                                    stats=stats)
        return res.stats if stats else None

    def run_all(stats=False, queries=None):
        return [run_wave(i, stats, queries) for i in range(len(waves))]

    if args.calib_copy:
        src_t = torch.ones(2**30 // 4, dtype=torch.float32, device="cuda:0")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src_t, dst_t

    tuning = None
    cache = None if args.retune else (TUNING_CACHE if os.path.exists(TUNING_CACHE) else None)
    if not args.no_autotune:
        sample = fora.make_queries(srcs[:min(32, WB)], alpha=alpha, eps=eps, k=k, seed=seed,
                                   n=g.n)
        rec = autotune.autotune(G, sample, path=cache, force=args.retune, log=log)
        tuning = dict(rec["tuning"])
        log(f"tuning ({'cached' if rec.get('cached') else 'measured'}): {tuning}")
    graph_rounds = G.get_tuning()["graph_rounds"]
    G.set_tuning(graph_rounds=0)  # timed region: host-driven rounds, per-phase events

    for i in range(args.warmup):
        run_wave(i % len(waves))
        log(f"warmup {i+1}/{args.warmup} done")
    torch.cuda.synchronize()
    step_times, walk_ms, stats_last = [], [], {}
    total_steps = total_walks = total_queries = total_edge_ops = 0
    ph_sum = dict(ms_push=0.0, ms_plan=0.0, ms_walk=0.0, ms_topk=0.0)
    t_all = time.perf_counter()
    for i in range(args.steps):
        wi = i % len(waves)
        ts = time.perf_counter()
        st = run_wave(wi, stats=True)
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - ts)
        stats_last[wi] = st
        total_steps += sum(s["steps"] for s in st)
        total_walks += sum(s["walks"] for s in st)
        total_edge_ops += sum(s["edge_ops"] for s in st)
        total_queries += len(st)
        for p in ph_sum:
            ph_sum[p] += st[0][p]
        walk_ms.append(st[0]["ms_walk"])
        log(f"step {i+1}/{args.steps} (wave {wi}): {step_times[-1]*1e3:.1f} ms "
            f"(push {st[0]['ms_push']:.1f} plan {st[0]['ms_plan']:.1f} "
            f"walk {st[0]['ms_walk']:.1f} topk {st[0]['ms_topk']:.1f})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    steps_per_s = total_steps / elapsed
    qps = total_queries / elapsed
    stats0 = stats_last[min(stats_last)]

    # the walk kernel against the HBM roofline: algorithmic bytes of the
    # timed launches over their HIP-event durations (one walk launch per step)
    per_launch_steps = total_steps / args.steps
    per_launch_walks = total_walks / args.steps
    walk_s = float(np.mean(walk_ms)) / 1e3
    alg_bytes = BYTES_PER_STEP * per_launch_steps + BYTES_PER_WALK * per_launch_walks
    achieved = alg_bytes / walk_s / 1e9
    traffic, traffic_src = recorded_traffic("k_walks", f"{args.workload}_b{WB}")
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS,
                    unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                    traffic_source=traffic_src, kernel="k_walks", bytes_per_launch=alg_bytes,
                    avg_launch_ms=round(walk_s * 1e3, 3))
    if traffic is not None:
        # the counters' HBM bytes per launch over this run's launch time: the
        # hardware rate, beside the algorithmic one above
        roofline["traffic_gbs"] = round(traffic / walk_s / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / walk_s / 1e9 / PEAK_HBM_GBS, 4)
    log(f"headline: {steps_per_s:.3e} walk-steps/s, {qps:.2f} q/s; walk kernel "
        f"{achieved:.0f} GB/s algorithmic ({achieved / PEAK_HBM_GBS:.1%})"
        + (f", {roofline['traffic_gbs']:.0f} GB/s by the counters "
           f"({roofline['traffic_frac']:.1%})" if traffic is not None else ""))

    def timed_leg(fn, steps):
        for i in range(leg_warmup):
            fn(i % len(waves))
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = [fn(i % len(waves)) for i in range(steps)]
        torch.cuda.synchronize()
        return time.perf_counter() - t, out

    learned_leg = None
    model_path = os.path.join(ROOT, "paper_1908_10583_amd", "models",
                              f"{args.workload}_rmax_mlp.json")
    if not args.no_learned and os.path.exists(model_path):
        from paper_1908_10583_amd import learned
        model = learned.Model.load(model_path)
        src_w = [torch.as_tensor(srcs[a:b], dtype=torch.int32, device="cuda:0")
                 for a, b in waves]

        def learned_wave(i):
            a, b = waves[i]
            rm, fb = model.predict_rmax(G, src_w[i], alpha, eps)
            q = fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n,
                                  rmax=rm.cpu().numpy())
            res = fora.fora_ssppr_batch(G, q, kmax=k, ws=ws, out=(ids[a:b], vals[a:b]),
                                        stats=True)
            return res.stats, fb

        dtl, outs = timed_leg(learned_wave, leg_steps)
        lq = sum(len(s) for s, _ in outs)
        l_steps = sum(x["steps"] for s, _ in outs for x in s)
        learned_leg = dict(queries_per_s=round(lq / dtl, 2), walk_steps_per_s=l_steps / dtl,
                           ms_per_step=round(dtl / leg_steps * 1e3, 3),
                           fallbacks=int(sum(fb for _, fb in outs)),
                           model=os.path.relpath(model_path, ROOT),
                           note="r_max per source from the BF16 MLP, inference inside the "
                                "timed step; the eps guarantee holds for any r_max (Lemma 2)")
        log(f"batched + learned r_max: {learned_leg['queries_per_s']} q/s")

    alg3 = None
    if not args.no_alg3:
        # Algorithm 3 (zero-hop pruning + push/walk balance): one walk's cost in
        # residue increments, the ratio of this GPU's marginal per-walk and
        # per-increment times (the rule weighs the walks still to come against
        # further pushing; averages over a whole query under-price walks), r_max
        # floor r_max* / 32 so that the balance rule ends the push
        from paper_1908_10583_amd import learned
        cal = learned.calibrate(G, srcs[:min(64, WB)], alpha=alpha, eps=eps)
        wc = cal["ms_per_walk"] / cal["ms_per_edge_op"]
        rstar = stats0[0]["rmax"]
        q3 = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n,
                                rmax=rstar / 32, flags=fora.FORA_PRUNE_ZERO_HOP |
                                fora.FORA_BALANCE, walk_cost=wc) for a, b in waves]
        dt3, outs = timed_leg(lambda i: run_wave(i, stats=True, queries=q3), leg_steps)
        st3 = [x for s in outs for x in s]
        alg3 = dict(queries_per_s=round(len(st3) / dt3, 2),
                    walk_steps_per_s=sum(x["steps"] for x in st3) / dt3,
                    ms_per_step=round(dt3 / leg_steps * 1e3, 3), walk_cost=round(wc, 3),
                    rmax_floor="r_max*/32",
                    balance_stopped=sum(x["balance_stopped"] for x in st3),
                    edge_ops=sum(x["edge_ops"] for x in st3),
                    walks=sum(x["walks"] for x in st3))
        log(f"Algorithm 3 (pruned + balanced, walk_cost {wc:.2f}): {alg3['queries_per_s']} q/s")

    index_leg = None
    if not args.no_index:
        # FORA+ (section 3.3): an index of omega_max(v) = ceil(d(v) r_max* omega_unit)
        # walk end points per node, built once; the timed queries read it
        rstar = stats0[0]["rmax"]
        wpd = rstar * stats0[0]["omega_unit"]
        torch.cuda.synchronize()
        tb = time.perf_counter()
        fora.fora_build_index(G, alpha, wpd, 0x5EED, seed)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - tb
        info = fora.fora_index_info(G)
        qi = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n,
                                flags=fora.FORA_USE_INDEX) for a, b in waves]
        dti, outs = timed_leg(lambda i: run_wave(i, stats=True, queries=qi), leg_steps)
        sti = [x for s in outs for x in s]
        index_leg = dict(queries_per_s=round(len(sti) / dti, 2),
                         ms_per_step=round(dti / leg_steps * 1e3, 3),
                         phases_ms={p: round(outs[-1][0][p], 3)
                                    for p in ("ms_push", "ms_plan", "ms_walk", "ms_topk")},
                         walks=sum(x["walks"] for x in sti),
                         live_walk_steps=sum(x["steps"] for x in sti),
                         index_entries=info["total"], index_bytes=info["total"] * 4 + 8 * (g.n + 1),
                         index_build_s=round(t_build, 3), walks_per_degree=wpd)
        log(f"FORA+ (index, built in {t_build:.2f}s, {info['total']} entries): "
            f"{index_leg['queries_per_s']} q/s")

    topk_leg = None
    if not args.no_topk:
        # top-k FORA (Algorithm 5): the same sources and k, eps and p_f of the
        # workload, delta halving from 1/k until the k-th estimate clears it
        qk = fora.make_queries(srcs[:WB], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n)
        outk = (ids[:len(qk)], vals[:len(qk)])
        dtk, outs = timed_leg(lambda i: fora.fora_topk_batch(G, qk, kmax=k, ws=ws, out=outk,
                                                             stats=True), leg_steps)
        rk, itk, dk = outs[-1]
        topk_leg = dict(queries_per_s=round(len(qk) * leg_steps / dtk, 2),
                        ms_per_step=round(dtk / leg_steps * 1e3, 3),
                        iterations_mean=float(np.mean(itk)),
                        final_delta_median=float(np.median(dk)),
                        walks=sum(x["walks"] for x in rk.stats),
                        note="approximate top-k (Definition 2) by Algorithm 5, not the "
                             "whole-graph query; sources of the first wave")
        log(f"top-k FORA (Algorithm 5): {topk_leg['queries_per_s']} q/s, "
            f"{topk_leg['iterations_mean']:.1f} iterations")

    pagerank_leg = None
    if not args.no_pagerank:
        # global PageRank: FORA from the source distribution (1/n, ..., 1/n),
        # the workload's eps, delta, p_f and k, one query per call
        dtp, outs = timed_leg(lambda i: fora.pagerank(G, alpha, eps, k=k, seed=seed, ws=ws,
                                                      stats=True), leg_steps)
        sp = outs[-1].stats
        pagerank_leg = dict(ms_per_query=round(dtp / leg_steps * 1e3, 3),
                            phases_ms={x: round(sp[x], 3) for x in
                                       ("ms_push", "ms_plan", "ms_walk", "ms_topk")},
                            rounds=sp["rounds"], edge_ops=sp["edge_ops"], walks=sp["walks"],
                            note="source distribution (1/n, ..., 1/n), the paper's "
                                 "extension of Algorithm 1")
        log(f"global PageRank: {pagerank_leg['ms_per_query']} ms per query")

    graph_mode = None
    if graph_rounds > 0 and not args.no_graph:
        G.set_tuning(graph_rounds=graph_rounds)
        run_wave(0)  # capture
        dtg, _ = timed_leg(lambda i: run_wave(i), leg_steps)
        gq = sum(waves[i % len(waves)][1] - waves[i % len(waves)][0] for i in range(leg_steps))
        graph_mode = dict(queries_per_s=round(gq / dtg, 2), graph_rounds=graph_rounds)
        log(f"graph replay: {gq / dtg:.1f} q/s")
        G.set_tuning(graph_rounds=0)

    single = None
    if not args.no_single:
        # the plain single-query loop runs in a launch shape tuned for one
        # query (the autotuner keys its cache by batch size), so that the
        # batching gain is measured against a tuned baseline
        saved_tuning = G.get_tuning()
        single_tuning = None
        if not args.no_autotune:
            one = fora.make_queries(srcs[:1], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n)
            single_tuning = dict(autotune.autotune(G, one, path=cache, force=args.retune,
                                                   log=log)["tuning"])
        ws1 = fora.workspace(G, 1)
        o1 = (torch.empty(k, dtype=torch.int32, device="cuda:0"),
              torch.empty(k, dtype=torch.float32, device="cuda:0"))
        fora.fora_ssppr(G, int(srcs[0]), alpha, eps, k=k, seed=seed, ws=ws1, out=o1)
        torch.cuda.synchronize()
        sample = srcs[:single_sample] if single_sample else srcs
        t1 = time.perf_counter()
        s_steps = 0
        for s in sample:
            r = fora.fora_ssppr(G, int(s), alpha, eps, k=k, seed=seed, ws=ws1, out=o1, stats=True)
            s_steps += r.stats["steps"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ns = len(sample)
        single = dict(queries_per_s=round(ns / dt, 2), walk_steps_per_s=s_steps / dt,
                      ms_per_query=round(dt / ns * 1e3, 3), sources=ns,
                      sample=f"the workload's first {ns} sources", tuning=single_tuning)
        log(f"plain single-query loop: {ns/dt:.1f} q/s over {ns} sources")
        del ws1
        G.set_tuning(**saved_tuning)

    small = None
    if not args.no_small:
        small = small_graph_leg(alpha, eps, k, seed, cache, args, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample)...")
        del ws
        cpu = cpu_baseline(g, srcs, alpha, eps, seed)
        log(f"cpu baseline: {cpu['value']:.3e} walk-steps/s on one core")

    workload = (f"{g.name}: {B} sources in {len(waves)} waves of {WB}, one wave per step"
                if multi else f"{g.name}, {B} sources, batched")
    out = {
        "metric": METRIC, "value": steps_per_s, "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "n": g.n, "m": g.m, "sources": B, "alpha": alpha,
                   "eps": eps, "delta": "1/n", "pf": "1/n", "k": k, "batch": WB,
                   "waves": len(waves)},
        "queries_per_s": round(qps, 2),
        "plain_single_query": single,
        "batched_vs_single": (round(qps / single["queries_per_s"], 3) if single else None),
        "batched_learned_rmax": learned_leg,
        "batched_alg3": alg3,
        "topk_fora": topk_leg,
        "global_pagerank": pagerank_leg,
        "fora_plus_index": index_leg,
        "graph_replay": graph_mode,
        "single_query_rmat20": small,
        "tuning": tuning,
        "phases_ms_per_step": {p: round(v / args.steps, 3) for p, v in ph_sum.items()},
        "per_step": {"walks": per_launch_walks, "walk_steps": per_launch_steps,
                     "edge_ops": total_edge_ops / args.steps,
                     "rounds_max": max(s["rounds"] for st in stats_last.values() for s in st)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
