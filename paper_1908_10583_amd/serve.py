"""Serving loop: Poisson arrivals, memory-based admission, continuous batching.

Requests (source, eps, k, seed) arrive over time and wait in one FIFO queue.
The server runs S slots, each a host thread with a HIP stream of its own.
A free slot takes the oldest waiting request together with the next waiting
requests of the same eps (so that one slow class does not hold up a batch of
fast queries), up to ``max_batch``, and only as many as the memory budget
admits: a batch of b queries needs the library's workspace for b queries
(dense per-query residue, reserve, walk counts, plan, frontiers), and the sum
over running batches never exceeds the budget. The batch then runs as one
``fora_ssppr_batch`` call on the slot's stream while other slots run theirs,
so requests that arrive while others are on the GPU are admitted as soon as
a slot and memory free up, and their device work overlaps.

Each query's result depends only on (graph, source, alpha, eps, delta, p_f,
k, r_max, seed): the push sums residues in fixed point (integer sums, the
same in any order) and walks are keyed by (source, seed, start node, walk
index), so a query returns the same result, bit for bit, alone or in any
batch.
"""
from __future__ import annotations

import collections
import json
import math
import threading
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import fora


@dataclass
class Request:
    id: int
    src: int
    eps: float
    k: int
    seed: int = 0
    rmax: float | None = None      # None: eqn:rmax (or the model's prediction)
    t_arrival: float = 0.0         # seconds on the server clock
    t_admit: float | None = None
    t_done: float | None = None
    slot: int = -1
    batch: int = 0
    ids: np.ndarray | None = None
    vals: np.ndarray | None = None
    stats: dict | None = None
    rows: dict | None = None       # copies of the dense rows (keep_rows=True)
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    """S slots over one graph. ``runner``/``ws_size`` can be replaced (host
    tests drive the scheduler without a GPU). ``query_flags`` go into every
    query (for example FORA_WALK_COUNTS, with ``keep_rows``, to inspect the
    per-node walk counts)."""

    def __init__(self, G, slots: int = 4, max_batch: int = 8, mem_budget: int | None = None,
                 alpha: float = 0.2, delta: float | None = None, pf: float | None = None,
                 model=None, keep_rows: bool = False, stats: bool = False,
                 ws_size=None, runner=None, query_flags: int = 0):
        if slots < 1 or max_batch < 1:
            raise ValueError("slots and max_batch must be at least 1")
        self.G = G
        self.alpha = alpha
        n = G.n if G is not None else 1
        self.delta = delta if delta is not None else 1.0 / n
        self.pf = pf if pf is not None else 1.0 / n
        self.slots = slots
        self.max_batch = max_batch
        self.model = model
        self.keep_rows = keep_rows
        self.want_stats = stats
        self.query_flags = int(query_flags)
        self.ws_size = ws_size or (lambda b: fora.fora_workspace_size(G, b))
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(G.device)
            mem_budget = int(0.85 * free)
        self.budget = int(mem_budget)
        if self.ws_size(1) > self.budget:
            raise ValueError(f"memory budget {self.budget} B is below one query's workspace "
                             f"({self.ws_size(1)} B)")
        self.runner = runner or self._run_batch
        self._own_streams = runner is None
        self.cv = threading.Condition()
        self.waiting: collections.deque[Request] = collections.deque()
        self.in_use = 0
        self.peak = 0
        self.running = 0
        self.max_running = 0
        self.batches = 0
        self.done: list[Request] = []
        self.closed = False
        self.t0 = time.perf_counter()
        self.workers = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                        for i in range(slots)]
        for w in self.workers:
            w.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ---------------------------------------------------------------- admission
    def submit(self, req: Request):
        with self.cv:
            if self.closed:
                raise RuntimeError("server is closed")
            self.waiting.append(req)
            self.cv.notify_all()

    def _take(self):
        """With the lock held: the oldest request and the following waiting
        requests of its eps, as many as max_batch and the memory budget allow."""
        head = self.waiting[0]
        picked = []
        for r in self.waiting:
            if r.eps == head.eps:
                picked.append(r)
                if len(picked) == self.max_batch:
                    break
        b = len(picked)
        while b > 0 and self.in_use + self.ws_size(b) > self.budget:
            b -= 1
        if b == 0:
            return None, 0
        picked = picked[:b]
        ids = {id(r) for r in picked}
        self.waiting = collections.deque(r for r in self.waiting if id(r) not in ids)
        nbytes = self.ws_size(b)
        self.in_use += nbytes
        self.peak = max(self.peak, self.in_use)
        return picked, nbytes

    def _worker(self, slot: int):
        stream = torch.cuda.Stream(device=self.G.device) if self._own_streams else None
        while True:
            with self.cv:
                while True:
                    if self.waiting:
                        batch, nbytes = self._take()
                        if batch:
                            break
                    elif self.closed:
                        return
                    self.cv.wait()
                t = self.now()
                for r in batch:
                    r.t_admit, r.slot, r.batch = t, slot, len(batch)
                self.running += 1
                self.batches += 1
                self.max_running = max(self.max_running, self.running)
            try:
                self.runner(batch, stream, nbytes)
            except Exception as e:  # the requests carry the error; the slot lives on
                for r in batch:
                    r.error = f"{type(e).__name__}: {e}"
            with self.cv:
                self.in_use -= nbytes
                self.running -= 1
                t = self.now()
                for r in batch:
                    r.t_done = t
                self.done.extend(batch)
                self.cv.notify_all()

    def close(self):
        """Stop admitting, finish what is queued, and join the slots."""
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()

    # ---------------------------------------------------------------- device work
    def _rmax_for(self, batch):
        rm = [r.rmax for r in batch]
        if self.model is None or not self.model.covers(self.alpha, batch[0].eps):
            return rm
        pred, _ = self.model.predict_rmax(self.G, [r.src for r in batch], self.alpha,
                                          batch[0].eps, self.delta, self.pf)
        pred = pred.cpu().numpy()
        return [r.rmax if r.rmax is not None else float(p) for r, p in zip(batch, pred)]

    def _run_batch(self, batch, stream, nbytes):
        G = self.G
        with torch.cuda.stream(stream):
            ws = torch.empty(nbytes, dtype=torch.uint8, device=G.device)
            qs = fora.make_queries([r.src for r in batch], alpha=self.alpha,
                                   eps=[r.eps for r in batch], delta=self.delta, pf=self.pf,
                                   k=[r.k for r in batch], rmax=self._rmax_for(batch),
                                   seed=[r.seed for r in batch], flags=self.query_flags)
            kmax = max(r.k for r in batch)
            res = fora.fora_ssppr_batch(G, qs, kmax=kmax, ws=ws, stats=self.want_stats,
                                        stream=stream)
            ids = res.ids.cpu().numpy()       # waits for the slot's stream
            vals = res.vals.cpu().numpy()
            rows = None
            if self.keep_rows:
                v = fora.fora_workspace_views(G, len(batch), ws)
                rows = {k: t.cpu().numpy() for k, t in v.items()}
            for i, r in enumerate(batch):
                r.ids = ids[i, :r.k].copy()
                r.vals = vals[i, :r.k].copy()
                if res.stats is not None:
                    r.stats = res.stats[i]
                if rows is not None:
                    r.rows = {k: a[i].copy() for k, a in rows.items()}
            del ws


def run_trace(server: Server, trace: list[dict], log=None) -> list[Request]:
    """Submits the requests of ``trace`` (dicts with id, t, src, eps, k, seed)
    at their arrival times on the server clock, waits for all of them and
    closes the server."""
    reqs = [Request(id=x["id"], src=x["src"], eps=x["eps"], k=x["k"], seed=x.get("seed", 0),
                    rmax=x.get("rmax")) for x in trace]
    start = server.now()
    last_log = time.perf_counter()
    for r, x in zip(reqs, trace):
        while True:
            d = start + x["t"] - server.now()
            if d <= 0:
                break
            time.sleep(min(d, 0.005))
        r.t_arrival = server.now()
        server.submit(r)
        if log and time.perf_counter() - last_log > 10:
            last_log = time.perf_counter()
            log(f"submitted {r.id + 1}/{len(reqs)}, done {len(server.done)}")
    while True:
        with server.cv:
            if len(server.done) == len(reqs):
                break
            server.cv.wait(timeout=10)
        if log:
            log(f"done {len(server.done)}/{len(reqs)}")
    server.close()
    return reqs


def summarize(reqs: list[Request], server: Server) -> dict:
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    wait = np.array([r.t_admit - r.t_arrival for r in ok]) * 1e3
    span = max(r.t_done for r in ok) - min(r.t_arrival for r in ok) if ok else float("nan")

    def pct(a, q):
        return float(np.percentile(a, q)) if a.size else float("nan")

    out = dict(requests=len(reqs), errors=len(reqs) - len(ok),
               queries_per_s=len(ok) / span if span > 0 else float("nan"),
               latency_ms=dict(p50=pct(lat, 50), p99=pct(lat, 99), mean=float(lat.mean())
                               if lat.size else float("nan")),
               queue_wait_ms=dict(p50=pct(wait, 50), p99=pct(wait, 99)),
               batches=server.batches, mean_batch=float(np.mean([r.batch for r in ok]))
               if ok else 0.0,
               max_concurrent_batches=server.max_running, peak_workspace_bytes=server.peak,
               budget_bytes=server.budget)
    by = {}
    for e in sorted({r.eps for r in ok}):
        le = np.array([r.latency for r in ok if r.eps == e]) * 1e3
        by[str(e)] = dict(count=int(le.size), p50=pct(le, 50), p99=pct(le, 99))
    out["latency_ms_by_eps"] = by
    errs = [r.error for r in reqs if r.error is not None]
    if errs:
        out["first_error"] = errs[0]
    return out


def main(argv=None):
    """Serves a Poisson trace of mixed-eps, mixed-k queries on a synthetic
    graph at one or more arrival rates; prints one JSON line per rate."""
    import argparse
    import sys

    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--qps", default="4", help="comma-separated arrival rates")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--mem-frac", type=float, default=0.85)
    ap.add_argument("--eps", default="0.1,0.5")
    ap.add_argument("--k", default="50,500")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--alone", type=int, default=8, help="requests also timed one at a time")
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    g, srcs = synth.workload(args.workload)
    log(f"graph {g.name} n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s")
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    del g
    eps_c = tuple(float(x) for x in args.eps.split(","))
    k_c = tuple(int(x) for x in args.k.split(","))
    per_query = fora.fora_workspace_size(G, 2) - fora.fora_workspace_size(G, 1)
    # warm-up: one query per eps class
    ws = fora.workspace(G, 1)
    for e in eps_c:
        fora.fora_ssppr(G, int(srcs[0]), eps=e, k=max(k_c), ws=ws)
    torch.cuda.synchronize()
    del ws
    # the same queries alone, one at a time, for reference latencies
    alone_trace = synth.poisson_requests(args.alone, 1.0, srcs, args.seed + 1, eps_c, k_c)
    alone_ms = {}
    for x in alone_trace:
        srv = Server(G, slots=1, max_batch=1, mem_budget=fora.fora_workspace_size(G, 1))
        r = run_trace(srv, [dict(x, t=0.0)])[0]
        alone_ms.setdefault(str(x["eps"]), []).append(r.latency * 1e3)
    if alone_ms:
        log(f"alone: {json.dumps({k: float(np.median(v)) for k, v in alone_ms.items()})}")
    free, total = torch.cuda.mem_get_info(G.device)
    budget = int(args.mem_frac * free)
    for qps in (float(x) for x in args.qps.split(",")):
        trace = synth.poisson_requests(args.requests, qps, srcs, args.seed, eps_c, k_c)
        srv = Server(G, slots=args.slots, max_batch=args.max_batch, mem_budget=budget)
        t1 = time.perf_counter()
        reqs = run_trace(srv, trace, log=log)
        rep = summarize(reqs, srv)
        rep.update(workload=args.workload, n=G.n, m=G.m, offered_qps=qps, slots=args.slots,
                   max_batch=args.max_batch, eps=list(eps_c), k=list(k_c),
                   workspace_bytes_per_query=per_query,
                   admission_cap_queries=int(budget // max(per_query, 1)),
                   alone_latency_ms={k: dict(p50=float(np.median(v)), count=len(v))
                                     for k, v in alone_ms.items()},
                   wall_s=time.perf_counter() - t1)
        print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
