"""Benchmark: FORA whole-graph SSPPR + top-500 on one MI355X.

Workload (default): R-MAT, 2^20 nodes, 16 * 2^20 samples (a, b, c) =
(.57, .19, .19), duplicates and self-loops removed, dangling nodes given one
random out-edge; 100 seeded sources uniform over nodes with R-MAT out-degree
>= 1; alpha = 0.2, eps = 0.5, delta = p_f = 1/n, k = 500.

One step = the whole hot path (push, walk plan, walks, estimate, top-k) for
all 100 sources in one batched call. The plain single-query loop over the
same sources is timed beside it. Prints one JSON line.
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def recorded_traffic(kernel: str, tag: str):
    """HBM-side bytes per launch from the committed counter record for this
    workload (tag: workload and batch, e.g. rmat20_b100), or None if there is
    none or the kernel's sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_{tag}_traffic.json")):
        rec = json.load(open(path))
        h = hashlib.sha256()
        try:
            for src in rec["sources"]:
                h.update(open(os.path.join(ROOT, src), "rb").read())
        except OSError:
            continue
        if h.hexdigest() == rec["source_sha256"]:
            return rec["traffic_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def cpu_baseline(g, src, alpha, eps, k, seed):
    import oracle
    t0 = time.perf_counter()
    out = oracle.fora(g, int(src), alpha=alpha, eps=eps, k=k, seed=seed)
    dt = time.perf_counter() - t0
    return dict(value=out["steps"] / dt, unit="walk-steps/s", cores=1, kind="oracle",
                queries_per_s=1.0 / dt, seconds=dt,
                sample=f"1 source (node {int(src)}) of the workload, full query, "
                       f"{out['steps']} walk steps, single-threaded FP64 C oracle")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--max-batch", type=int, default=0,
                    help="queries per batched call (0: all sources in one call)")
    ap.add_argument("--single-sample", type=int, default=0,
                    help="sources timed by the plain single-query loop (0: all)")
    ap.add_argument("--sources", type=int, default=0,
                    help="use only the workload's first N sources (0: all)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--no-alg3", action="store_true", help="skip the Algorithm 3 leg")
    ap.add_argument("--no-topk", action="store_true", help="skip the top-k FORA leg")
    ap.add_argument("--no-pagerank", action="store_true", help="skip the global PageRank leg")
    ap.add_argument("--no-index", action="store_true", help="skip the FORA+ (index) leg")
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
    # the sources run in waves of at most --max-batch queries (per-query
    # state is dense, so large graphs take several waves)
    WB = min(B, args.max_batch) if args.max_batch else B
    waves = [(a, min(a + WB, B)) for a in range(0, B, WB)]
    qs_w = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n)
            for a, b in waves]
    ws_bytes = fora.fora_workspace_size(G, WB)
    if not args.no_topk:  # the top-k leg reuses it (staging rows after the main layout)
        ws_bytes = max(ws_bytes, fora.fora_topk_workspace_size(G, WB, k))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    ids = torch.empty((B, k), dtype=torch.int32, device="cuda:0")
    vals = torch.empty((B, k), dtype=torch.float32, device="cuda:0")
    log(f"workspace {ws.numel()/2**30:.2f} GiB for waves of {WB} ({len(waves)} waves)")

    def run_all(stats=False, queries=None):
        out = []
        for i, (a, b) in enumerate(waves):
            q = qs_w[i] if queries is None else queries[i]
            res = fora.fora_ssppr_batch(G, q, kmax=k, ws=ws, out=(ids[a:b], vals[a:b]),
                                        stats=stats)
            if stats:
                out.append(res.stats)
        return out

    if args.calib_copy:
        src_t = torch.ones(2**30 // 4, dtype=torch.float32, device="cuda:0")
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src_t, dst_t

    tuning = None
    if not args.no_autotune:
        sample = fora.make_queries(srcs[:min(32, WB)], alpha=alpha, eps=eps, k=k, seed=seed,
                                   n=g.n)
        rec = autotune.autotune(G, sample, log=log)
        tuning = dict(rec["tuning"])
    graph_rounds = G.get_tuning()["graph_rounds"]
    G.set_tuning(graph_rounds=0)  # timed region: host-driven rounds, per-phase events

    for i in range(args.warmup):
        run_all()
        log(f"warmup {i+1}/{args.warmup} done")
    torch.cuda.synchronize()
    step_times, walk_ms, stats0 = [], [], None
    total_steps = total_walks = 0
    t_all = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        per_wave = run_all(stats=True)
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - ts)
        st = [x for w in per_wave for x in w]
        stats0 = st
        total_steps += sum(s["steps"] for s in st)
        total_walks += sum(s["walks"] for s in st)
        ph = {p: sum(w[0][p] for w in per_wave) for p in ("ms_push", "ms_plan", "ms_walk",
                                                           "ms_topk")}
        walk_ms.append(ph["ms_walk"] / len(waves))
        log(f"step {i+1}/{args.steps}: {step_times[-1]*1e3:.1f} ms "
            f"(push {ph['ms_push']:.1f} plan {ph['ms_plan']:.1f} "
            f"walk {ph['ms_walk']:.1f} topk {ph['ms_topk']:.1f})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    steps_per_s = total_steps / elapsed
    qps = B * args.steps / elapsed

    per_launch_steps = total_steps / args.steps / len(waves)
    per_launch_walks = total_walks / args.steps / len(waves)
    walk_s = float(np.mean(walk_ms)) / 1e3
    alg_bytes = BYTES_PER_STEP * per_launch_steps + BYTES_PER_WALK * per_launch_walks
    achieved = alg_bytes / walk_s / 1e9
    traffic, traffic_src = recorded_traffic("k_walks", f"{args.workload}_b{WB}")
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS,
                    unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                    traffic_source=traffic_src, kernel="k_walks", bytes_per_launch=alg_bytes,
                    avg_launch_ms=round(walk_s * 1e3, 3))

    learned_leg = None
    model_path = os.path.join(ROOT, "paper_1908_10583_amd", "models",
                              f"{args.workload}_rmax_mlp.json")
    if not args.no_learned and os.path.exists(model_path):
        from paper_1908_10583_amd import learned
        model = learned.Model.load(model_path)
        src_t = torch.as_tensor(srcs, dtype=torch.int32, device="cuda:0")

        def learned_step(stats=False):
            rm, fb = model.predict_rmax(G, src_t, alpha, eps)
            rm = rm.cpu().numpy()
            q_l = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n,
                                     rmax=rm[a:b]) for a, b in waves]
            return run_all(stats=stats, queries=q_l), fb

        for _ in range(args.warmup):
            learned_step()
        torch.cuda.synchronize()
        tl = time.perf_counter()
        l_steps = 0
        for _ in range(args.steps):
            per_wave, fb = learned_step(stats=True)
            l_steps += sum(s["steps"] for w in per_wave for s in w)
        torch.cuda.synchronize()
        dtl = time.perf_counter() - tl
        learned_leg = dict(queries_per_s=round(B * args.steps / dtl, 2),
                           walk_steps_per_s=l_steps / dtl,
                           ms_per_step=round(dtl / args.steps * 1e3, 3), fallbacks=fb,
                           model=os.path.relpath(model_path, ROOT),
                           note="r_max per source from the BF16 MLP, inference inside the "
                                "timed step; the eps guarantee holds for any r_max (Lemma 2)")
        log(f"batched + learned r_max: {B * args.steps / dtl:.1f} q/s")

    alg3 = None
    if not args.no_alg3:
        # Algorithm 3 (zero-hop pruning + push/walk balance): one walk's cost in
        # residue increments, the ratio of this GPU's marginal per-walk and
        # per-increment times (the rule weighs the walks still to come against
        # further pushing; averages over a whole query under-price walks), r_max
        # floor r_max* / 32 so that the balance rule ends the push
        from paper_1908_10583_amd import learned
        cal = learned.calibrate(G, srcs[:min(64, B)], alpha=alpha, eps=eps)
        wc = cal["ms_per_walk"] / cal["ms_per_edge_op"]
        rstar = stats0[0]["rmax"]
        q3 = [fora.make_queries(srcs[a:b], alpha=alpha, eps=eps, k=k, seed=seed, n=g.n,
                                rmax=rstar / 32, flags=fora.FORA_PRUNE_ZERO_HOP |
                                fora.FORA_BALANCE, walk_cost=wc) for a, b in waves]
        for _ in range(args.warmup):
            run_all(queries=q3)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        a_steps = 0
        for _ in range(args.steps):
            pw3 = run_all(stats=True, queries=q3)
            a_steps += sum(x["steps"] for w in pw3 for x in w)
        torch.cuda.synchronize()
        dt3 = time.perf_counter() - t3
        st3 = [x for w in pw3 for x in w]
        alg3 = dict(queries_per_s=round(B * args.steps / dt3, 2), walk_steps_per_s=a_steps / dt3,
                    ms_per_step=round(dt3 / args.steps * 1e3, 3), walk_cost=round(wc, 3),
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
        for _ in range(args.warmup):
            run_all(queries=qi)
        torch.cuda.synchronize()
        ti = time.perf_counter()
        for _ in range(args.steps):
            pwi = run_all(stats=True, queries=qi)
        torch.cuda.synchronize()
        dti = time.perf_counter() - ti
        sti = [x for w in pwi for x in w]
        index_leg = dict(queries_per_s=round(B * args.steps / dti, 2),
                         ms_per_step=round(dti / args.steps * 1e3, 3),
                         phases_ms={p: round(sum(w[0][p] for w in pwi), 3)
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
        wsk = ws  # sized for both at the start (one workspace of this size fits in HBM)
        outk = (ids[:len(qk)], vals[:len(qk)])
        for _ in range(args.warmup):
            fora.fora_topk_batch(G, qk, kmax=k, ws=wsk, out=outk)
        torch.cuda.synchronize()
        tk = time.perf_counter()
        for _ in range(args.steps):
            rk, itk, dk = fora.fora_topk_batch(G, qk, kmax=k, ws=wsk, out=outk, stats=True)
        torch.cuda.synchronize()
        dtk = time.perf_counter() - tk
        topk_leg = dict(queries_per_s=round(len(qk) * args.steps / dtk, 2),
                        ms_per_step=round(dtk / args.steps * 1e3, 3),
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
        fora.pagerank(G, alpha, eps, k=k, seed=seed, ws=ws)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.steps):
            rp = fora.pagerank(G, alpha, eps, k=k, seed=seed, ws=ws, stats=True)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        sp = rp.stats
        pagerank_leg = dict(ms_per_query=round(dtp / args.steps * 1e3, 3),
                            phases_ms={x: round(sp[x], 3) for x in
                                       ("ms_push", "ms_plan", "ms_walk", "ms_topk")},
                            rounds=sp["rounds"], edge_ops=sp["edge_ops"], walks=sp["walks"],
                            note="source distribution (1/n, ..., 1/n), the paper's "
                                 "extension of Algorithm 1")
        log(f"global PageRank: {pagerank_leg['ms_per_query']} ms per query")

    graph_mode = None
    if graph_rounds > 0 and not args.no_graph:
        G.set_tuning(graph_rounds=graph_rounds)
        run_all()  # capture
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            run_all()
        torch.cuda.synchronize()
        dtg = time.perf_counter() - tg
        graph_mode = dict(queries_per_s=round(B * args.steps / dtg, 2),
                          walk_steps_per_s=total_steps / dtg, graph_rounds=graph_rounds)
        log(f"graph replay: {B * args.steps / dtg:.1f} q/s")
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
            single_tuning = dict(autotune.autotune(G, one, log=log)["tuning"])
        ws1 = fora.workspace(G, 1)
        o1 = (torch.empty(k, dtype=torch.int32, device="cuda:0"),
              torch.empty(k, dtype=torch.float32, device="cuda:0"))
        fora.fora_ssppr(G, int(srcs[0]), alpha, eps, k=k, seed=seed, ws=ws1, out=o1)
        torch.cuda.synchronize()
        sample = srcs[:args.single_sample] if args.single_sample else srcs
        t1 = time.perf_counter()
        s_steps = 0
        for s in sample:
            r = fora.fora_ssppr(G, int(s), alpha, eps, k=k, seed=seed, ws=ws1, out=o1, stats=True)
            s_steps += r.stats["steps"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ns = len(sample)
        single = dict(queries_per_s=round(ns / dt, 2), walk_steps_per_s=s_steps / dt,
                      ms_per_query=round(dt / ns * 1e3, 3), sources=ns, tuning=single_tuning)
        log(f"plain single-query loop: {ns/dt:.1f} q/s over {ns} sources")
        del ws1
        G.set_tuning(**saved_tuning)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one source)...")
        cpu = cpu_baseline(g, srcs[0], alpha, eps, k, seed)
        log(f"cpu baseline: {cpu['seconds']:.1f}s")

    out = {
        "metric": METRIC, "value": steps_per_s, "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{g.name}, {B} sources, batched", "n": g.n, "m": g.m,
                   "sources": B, "alpha": alpha, "eps": eps, "delta": "1/n", "pf": "1/n",
                   "k": k, "batch": WB, "waves": len(waves)},
        "queries_per_s": round(qps, 2),
        "plain_single_query": single,
        "batched_learned_rmax": learned_leg,
        "batched_alg3": alg3,
        "topk_fora": topk_leg,
        "global_pagerank": pagerank_leg,
        "fora_plus_index": index_leg,
        "graph_replay": graph_mode,
        "tuning": tuning,
        "phases_ms": {p: round(float(v), 3) for p, v in ph.items()},
        "per_step": {"walks": per_launch_walks, "walk_steps": per_launch_steps,
                     "edge_ops": sum(s["edge_ops"] for s in stats0),
                     "rounds_max": max(s["rounds"] for s in stats0)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
