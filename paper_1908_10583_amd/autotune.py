"""Autotuner for the library's launch shape (``fora_tuning``).

It times real batched calls on the caller's graph and queries with the
library's own per-phase HIP-event timers, picks the fastest shape phase by
phase (pull/push switch point, push grid, then walk grid x walk chunk x
end-point aggregation), decides whether replaying a
captured HIP graph beats the host-driven push loop, and caches the result in
a JSON file keyed by device, graph size and batch size. Results never depend
on the tuning; only speed does.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import fora

PULL_RATIOS = (0, 4, 16, 64, 256)
PUSH_BLOCKS = (2, 4, 8, 16, 32)
WALK_BLOCKS = (2, 4, 8, 12, 16)
WALK_CHUNKS = (256, 512, 1024, 2048, 4096)
WALK_AGG = (0, 1)


def cache_path() -> str:
    return os.environ.get("FORA_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fora", "tuning.json"))


def _key(G: fora.Graph, batch: int) -> str:
    props = torch.cuda.get_device_properties(G.device)
    bucket = 1 << max(0, (batch - 1).bit_length())
    # the architecture name, not the marketing name (which some tools blank)
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch}|cu={props.multi_processor_count}|n={G.n}|m={G.m}|batch<={bucket}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _timed(G, queries, ws, out, reps=2):
    """Best-of-reps phase times (ms) and wall time of one batched call."""
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fora.fora_ssppr_batch(G, queries, ws=ws, out=out, stats=True)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        st = res.stats[0]
        cur = dict(push=st["ms_push"], walk=st["ms_walk"], wall=wall,
                   rounds=max(s["rounds"] for s in res.stats))
        if best is None or cur["wall"] < best["wall"]:
            best = cur
    return best


def autotune(G: fora.Graph, queries, path: str | None = None, force: bool = False,
             log=None) -> dict:
    """Tune ``G`` for batches like ``queries`` (a fora_query array); returns the
    chosen tuning (also applied to ``G``) with the measurements behind it."""
    path = path or cache_path()
    key = _key(G, len(queries))
    cache = _load(path)
    if not force and key in cache:
        t = cache[key]["tuning"]
        G.set_tuning(**t)
        return dict(cache[key], cached=True)
    B = len(queries)
    kmax = max(q.k for q in queries)
    ws = fora.workspace(G, B)
    out = (torch.empty((B, kmax), dtype=torch.int32, device=G.device),
           torch.empty((B, kmax), dtype=torch.float32, device=G.device))
    # record_ids stays 1: ids in the walk-record slots where they fit save a
    # line read per walk and never cost one
    base = dict(walk_blocks_per_cu=8, walk_chunk=512, push_blocks_per_cu=4, graph_rounds=0,
                pull_ratio=16, record_ids=1)
    G.set_tuning(**base)
    _timed(G, queries, ws, out, reps=1)  # warm-up
    trials = []
    best_ratio = None
    for pr in PULL_RATIOS:
        G.set_tuning(**dict(base, pull_ratio=pr))
        m = _timed(G, queries, ws, out)
        trials.append(dict(pull_ratio=pr, **m))
        if best_ratio is None or m["push"] < best_ratio[1]:
            best_ratio = (pr, m["push"])
    base["pull_ratio"] = best_ratio[0]
    if log:
        log(f"autotune: pull_ratio {best_ratio[0]} (push {best_ratio[1]:.2f} ms)")
    best_push = None
    for pb in PUSH_BLOCKS:
        G.set_tuning(**dict(base, push_blocks_per_cu=pb))
        m = _timed(G, queries, ws, out)
        trials.append(dict(push_blocks_per_cu=pb, **m))
        if best_push is None or m["push"] < best_push[1]:
            best_push = (pb, m["push"], m["rounds"])
    base["push_blocks_per_cu"] = best_push[0]
    if log:
        log(f"autotune: push_blocks_per_cu {best_push[0]} (push {best_push[1]:.2f} ms)")
    best_walk = None
    for agg in WALK_AGG:
        if log:
            log(f"autotune: walk shapes with walk_agg={agg}")
        for wb in WALK_BLOCKS:
            for ch in WALK_CHUNKS:
                G.set_tuning(**dict(base, walk_blocks_per_cu=wb, walk_chunk=ch, walk_agg=agg))
                m = _timed(G, queries, ws, out)
                trials.append(dict(walk_blocks_per_cu=wb, walk_chunk=ch, walk_agg=agg, **m))
                if best_walk is None or m["walk"] < best_walk[2]:
                    best_walk = (wb, ch, m["walk"], agg)
    base["walk_blocks_per_cu"], base["walk_chunk"] = best_walk[0], best_walk[1]
    base["walk_agg"] = best_walk[3]
    G.set_tuning(**base)
    eager = _timed(G, queries, ws, out, reps=3)
    rounds = int(best_push[2] * 1.25) + 4
    G.set_tuning(**dict(base, graph_rounds=rounds))
    _timed(G, queries, ws, out, reps=1)  # capture
    graph = _timed(G, queries, ws, out, reps=3)
    use_graph = graph["wall"] < eager["wall"]
    tuning = dict(base, graph_rounds=rounds if use_graph else 0)
    G.set_tuning(**tuning)
    rec = dict(tuning=tuning, eager_ms=eager["wall"], graph_ms=graph["wall"],
               push_ms=best_push[1], walk_ms=best_walk[2], trials=trials,
               measured_batch=B, time=time.time())
    cache[key] = rec
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    if log:
        log(f"autotune {key}: {tuning} (eager {eager['wall']:.2f} ms, graph {graph['wall']:.2f} ms)")
    return dict(rec, cached=False)
