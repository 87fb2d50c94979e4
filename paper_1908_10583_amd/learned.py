"""Learned per-source r_max.

For each training source the library pushes once through 16 thresholds
r_i = mult_i * r_max* (mult from 8 down to 1/32, log-spaced; each threshold
continues from the previous one's state) and records the exact push work
E_i (residue increments) and the walk count W_i Algorithm 2 would then run.
Costs are priced with marginal per-unit push and walk times measured on this
GPU (the slopes of each phase's time against its work over batched FORA
calls at several r_max, timed by the library's phase events), so
label(s) = ln(mult of the cheapest threshold). A 7 -> 64 -> 64 -> 1 GELU MLP
is trained on (features, label) with the library's own forward, backward and
Adam kernels; inference runs the library's BF16 kernel, which maps the
output y to r_max = r_max* exp(y) and falls back to r_max* for outputs that
are not finite or leave the trained range. Since Lemma 2 holds for any
r_max, the eps guarantee is unaffected; only cost changes.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import fora

MULTS = np.exp(np.linspace(math.log(8.0), math.log(1.0 / 32), 16))  # descending
LOG_LO, LOG_HI = math.log(1.0 / 32), math.log(8.0)
# the output range of models saved before the grid reached below 0.25 r_max*
LEGACY_LOG_RANGE = (math.log(0.25), math.log(8.0))


def features(G, srcs, alpha=0.2, eps=0.5, delta=None, pf=None):
    delta = 1.0 / G.n if delta is None else delta
    pf = 1.0 / G.n if pf is None else pf
    return fora.fora_features(G, torch.as_tensor(np.asarray(srcs), dtype=torch.int32),
                              alpha, eps, delta, pf)


def sweep(G, srcs, alpha=0.2, eps=0.5, delta=None, pf=None, batch=128, log=None):
    """Push work E[s, i] and walk counts W[s, i] at every threshold of MULTS."""
    srcs = np.asarray(srcs)
    E = np.zeros((len(srcs), len(MULTS)), np.int64)
    W = np.zeros((len(srcs), len(MULTS)), np.uint64)
    ws = fora.workspace(G, batch)
    t0 = time.perf_counter()
    for i in range(0, len(srcs), batch):
        part = srcs[i:i + batch]
        qs = fora.make_queries(part, alpha=alpha, eps=eps, delta=delta, pf=pf, k=1, n=G.n)
        e, w = fora.fora_push_sweep(G, qs, MULTS, ws=ws)
        E[i:i + len(part)] = e
        W[i:i + len(part)] = w
        if log and (i // batch) % 2 == 0:
            log(f"sweep {i + len(part)}/{len(srcs)} ({time.perf_counter() - t0:.1f}s)")
    return E, W


def calibrate(G, srcs, alpha=0.2, eps=0.5, mults=(1 / 32, 1 / 8, 0.5, 1.0, 2.0, 8.0),
              batch=64):
    """Marginal per-unit costs on this GPU: ms per residue increment (push)
    and ms per walk, the slopes of affine least-squares fits of each phase's
    time against its work over batched FORA calls at several r_max
    multipliers (the intercepts take the per-call and per-round overheads,
    which do not scale with the work)."""
    srcs = np.asarray(srcs)[:batch]
    ws = fora.workspace(G, len(srcs))
    fora.fora_ssppr_batch(G, fora.make_queries(srcs, alpha=alpha, eps=eps, k=1, n=G.n), ws=ws)
    c = fora.fora_ssppr_batch(G, fora.make_queries(srcs[:1], alpha=alpha, eps=eps, k=1, n=G.n),
                              ws=ws, stats=True).stats[0]
    rstar = c["rmax"]
    rows = []
    for mlt in mults:
        qs = fora.make_queries(srcs, alpha=alpha, eps=eps, k=1, n=G.n, rmax=rstar * mlt)
        for _ in range(2):  # the second call is the one kept (warm)
            st = fora.fora_ssppr_batch(G, qs, ws=ws, stats=True).stats
        rows.append((st[0]["ms_push"], st[0]["ms_walk"], sum(s["edge_ops"] for s in st),
                     sum(s["walks"] for s in st)))
    r = np.asarray(rows, np.float64)

    def slope(t, x):
        A = np.stack([x, np.ones_like(x)], 1)
        return float(np.linalg.lstsq(A, t, rcond=None)[0][0])

    a = slope(r[:, 0], r[:, 2])
    b = slope(r[:, 1], r[:, 3])
    # a fit with a non-positive slope (noise) falls back to the average cost
    a = a if a > 0 else float(r[:, 0].sum() / max(r[:, 2].sum(), 1.0))
    b = b if b > 0 else float(r[:, 1].sum() / max(r[:, 3].sum(), 1.0))
    return dict(ms_per_edge_op=a, ms_per_walk=b, rmax_star=rstar,
                calibration=dict(mults=list(map(float, mults)), rows=r.tolist()))


def labels(E, W, cost):
    """Per-source label ln(mult) at the modelled cost minimum: the grid's
    argmin refined by the vertex of the parabola through it and its two grid
    neighbours (the grid is uniform in ln mult), kept within the grid."""
    total = cost["ms_per_edge_op"] * E.astype(np.float64) + \
        cost["ms_per_walk"] * W.astype(np.float64)
    x = np.log(MULTS)
    h = x[1] - x[0]
    best = np.argmin(total, axis=1)
    y = x[best].copy()
    inner = (best > 0) & (best < len(MULTS) - 1)
    rows = np.flatnonzero(inner)
    cm = total[rows, best[rows] - 1]
    c0 = total[rows, best[rows]]
    cp = total[rows, best[rows] + 1]
    curv = cm - 2.0 * c0 + cp
    ok = curv > 0
    off = np.zeros(rows.size)
    off[ok] = 0.5 * (cm[ok] - cp[ok]) / curv[ok]
    y[rows] += np.clip(off, -0.5, 0.5) * h
    return y, total


class Model:
    """MLP parameters on the device (FP32 master copy, BF16 inference copy)."""

    def __init__(self, params: torch.Tensor, trained_on=((0.2, 0.5),),
                 log_range=(LOG_LO, LOG_HI)):
        self.params = params
        # the (alpha, eps) pairs of the training set; other queries keep eqn:rmax
        self.trained_on = [tuple(map(float, x)) for x in trained_on]
        # the label grid's range in ln(r_max / r_max*): predictions outside
        # it fall back to eqn:rmax
        self.log_range = tuple(map(float, log_range))

    def covers(self, alpha: float, eps: float) -> bool:
        return any(abs(alpha - a) < 1e-12 and abs(eps - e) < 1e-12 for a, e in self.trained_on)

    @classmethod
    def init(cls, X: np.ndarray, seed=0, device="cuda"):
        rng = np.random.default_rng(seed)
        p = np.zeros(fora.FORA_MLP_PARAMS, np.float32)
        X = np.asarray(X, np.float64)
        mu = X.mean(0)
        sd = X.std(0)
        # features constant over the training set (ln n, ln m, alpha, eps on
        # one graph) keep sigma = 1: a tiny sigma would blow up the BF16
        # rounding of mu at inference
        sd[sd < 1e-3 * np.maximum(1.0, np.abs(mu))] = 1.0
        p[0:7], p[7:14] = mu, sd
        o = 14
        for fan_in, fan_out in ((7, 64), (64, 64), (64, 1)):
            lim = math.sqrt(6.0 / (fan_in + fan_out))
            p[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
            o += fan_in * fan_out + fan_out  # biases stay 0
        return cls(torch.from_numpy(p).to(device))

    def train(self, X, y, epochs=300, lr=3e-3, batch=1024, seed=0, log=None):
        self._pb = None
        dev = self.params.device
        Xt = torch.as_tensor(np.asarray(X, np.float32), device=dev)
        yt = torch.as_tensor(np.asarray(y, np.float32), device=dev)
        N = Xt.shape[0]
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        grad = torch.zeros_like(self.params)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        acts = torch.empty((batch, fora.FORA_MLP_ACTS), dtype=torch.float32, device=dev)
        scratch = torch.empty(fora.FORA_MLP_SCRATCH(batch), dtype=torch.float32, device=dev)
        g = torch.Generator(device="cpu").manual_seed(seed)
        step = 0
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(dev)
            tot = 0.0
            for i in range(0, N - batch + 1 if N >= batch else 1, batch):
                idx = perm[i:i + batch]
                xb = Xt[idx].contiguous()
                yb = yt[idx].contiguous()
                yp = fora.fora_mlp_forward(xb, self.params, acts[:xb.shape[0]])
                fora.fora_mlp_backward(xb, self.params, acts[:xb.shape[0]], yp, yb, grad, loss,
                                       scratch)
                step += 1
                fora.fora_adam_step(self.params, grad, m, v, lr, 0.9, 0.999, 1e-8, step)
                tot += float(loss.item()) if (i == 0) else 0.0
            hist.append(tot)
            if log and ep % 50 == 0:
                log(f"epoch {ep}: batch loss {tot:.4f}")
        return hist

    def mse(self, X, y):
        Xt = torch.as_tensor(np.asarray(X, np.float32), device=self.params.device)
        yp = fora.fora_mlp_forward(Xt, self.params).cpu().numpy()
        return float(np.mean((yp - np.asarray(y)) ** 2))

    def bf16(self):
        """The BF16 inference copy (made once per set of trained weights)."""
        if getattr(self, "_pb", None) is None:
            self._pb = fora.fora_mlp_to_bf16(self.params)
        return self._pb

    def predict_rmax(self, G, srcs, alpha=0.2, eps=0.5, delta=None, pf=None):
        delta = 1.0 / G.n if delta is None else delta
        pf = 1.0 / G.n if pf is None else pf
        if not torch.is_tensor(srcs):
            srcs = torch.as_tensor(np.asarray(srcs), dtype=torch.int32)
        return fora.fora_predict_rmax(G, srcs, self.bf16(), alpha, eps, delta, pf,
                                      *self.log_range)

    def save(self, path):
        with open(path, "w") as f:
            json.dump(dict(params=self.params.cpu().numpy().tolist(),
                           trained_on=self.trained_on, log_range=self.log_range), f)

    @classmethod
    def load(cls, path, device="cuda"):
        with open(path) as f:
            d = json.load(f)
        p = np.asarray(d["params"], np.float32)
        return cls(torch.from_numpy(p).to(device), d.get("trained_on", ((0.2, 0.5),)),
                   d.get("log_range", LEGACY_LOG_RANGE))


def time_queries(G, srcs, rmax=None, alpha=0.2, eps=0.5, k=500):
    """Per-query wall time (ms) of single fora_ssppr calls."""
    ws = fora.workspace(G, 1)
    out = (torch.empty(k, dtype=torch.int32, device=G.device),
           torch.empty(k, dtype=torch.float32, device=G.device))
    fora.fora_ssppr(G, int(srcs[0]), alpha, eps, k=k, ws=ws, out=out)
    t = np.zeros(len(srcs))
    for i, s in enumerate(srcs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fora.fora_ssppr(G, int(s), alpha, eps, k=k, ws=ws, out=out,
                        rmax=None if rmax is None else float(rmax[i]))
        torch.cuda.synchronize()
        t[i] = (time.perf_counter() - t0) * 1e3
    return t


def time_batched(G, srcs, rmax=None, alpha=0.2, eps=0.5, k=500, batch=128):
    """Queries per second of batched calls over all sources."""
    ws = fora.workspace(G, batch)
    total = 0.0
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(0, len(srcs), batch):
            part = srcs[i:i + batch]
            rm = None if rmax is None else rmax[i:i + batch]
            qs = fora.make_queries(part, alpha=alpha, eps=eps, k=k, n=G.n, rmax=rm)
            fora.fora_ssppr_batch(G, qs, ws=ws)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0  # keep the second (warm) pass
    return len(srcs) / total


def main(argv=None):
    """Train on a workload's training sources and evaluate on its held-out
    sources against the fixed eqn:rmax rule; prints one JSON report.

    The cost sweep can run in pieces: ``--sweep-range a:b --sweep-dir D``
    sweeps training sources a..b-1 (plus the unit-cost calibration when
    a = 0) into D; a later call with ``--sweep-dir D`` and no range trains
    and evaluates from what D holds, sweeping whatever is missing."""
    import argparse
    import os
    import sys

    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--heldout", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--timed", type=int, default=512, help="held-out sources timed one by one")
    ap.add_argument("--sweep-batch", type=int, default=128)
    ap.add_argument("--sweep-dir", default=None)
    ap.add_argument("--sweep-range", default=None, help="a:b, sweep only these training sources")
    ap.add_argument("--model-out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[learned] {msg}", file=sys.stderr, flush=True)

    g, srcs = synth.workload(args.workload)
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    tr, ho = srcs[:args.train], srcs[-args.heldout:]
    assert len(srcs) >= args.train + args.heldout, "training and held-out sources overlap"
    log(f"graph {g.name} n={g.n} m={g.m}; train {len(tr)} held-out {len(ho)}")
    sd = args.sweep_dir
    if sd:
        os.makedirs(sd, exist_ok=True)

    def piece_path(a, b):
        return os.path.join(sd, f"{args.workload}_sweep_{a}_{b}.npz")

    def run_piece(a, b):
        t0 = time.perf_counter()
        E, W = sweep(G, tr[a:b], batch=args.sweep_batch, log=log)
        log(f"swept {a}:{b} in {time.perf_counter() - t0:.1f}s")
        if sd:
            np.savez(piece_path(a, b), E=E, W=W, srcs=tr[a:b])
        return E, W

    cost_path = os.path.join(sd, f"{args.workload}_unit_costs.json") if sd else None
    if cost_path and os.path.exists(cost_path):
        cost = json.load(open(cost_path))
    else:
        cost = calibrate(G, tr)
        if cost_path:
            json.dump(cost, open(cost_path, "w"))
    log(f"unit costs {cost}")
    if args.sweep_range:
        # saved in pieces of 1024 sources, so that a cut-off run keeps its work
        a, b = (int(x) for x in args.sweep_range.split(":"))
        b = min(b, len(tr))
        for lo in range(a, b, 1024):
            run_piece(lo, min(lo + 1024, b))
        return None

    # assemble the training sweep from saved pieces, sweeping the gaps
    E = np.zeros((len(tr), len(MULTS)), np.int64)
    W = np.zeros((len(tr), len(MULTS)), np.uint64)
    have = np.zeros(len(tr), bool)
    t_sweep0 = time.perf_counter()
    if sd:
        for f in sorted(os.listdir(sd)):
            if f.startswith(f"{args.workload}_sweep_") and f.endswith(".npz"):
                a, b = (int(x) for x in f[:-4].split("_")[-2:])
                z = np.load(os.path.join(sd, f), allow_pickle=False)
                # pieces of another threshold grid are swept again
                if b <= len(tr) and np.array_equal(z["srcs"], tr[a:b]) and \
                        z["E"].shape[1] == len(MULTS):
                    E[a:b], W[a:b], have[a:b] = z["E"], z["W"], True
    for a in range(0, len(tr), 1024):
        b = min(a + 1024, len(tr))
        if not have[a:b].all():
            E[a:b], W[a:b] = run_piece(a, b)
    t_sweep = time.perf_counter() - t_sweep0
    y, _ = labels(E, W, cost)
    X = features(G, tr).cpu().numpy()
    model = Model.init(X, seed=0)
    t1 = time.perf_counter()
    model.train(X, y, epochs=args.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    if args.model_out:
        model.save(args.model_out)
    Eh, Wh = sweep(G, ho, batch=args.sweep_batch)
    yh, cost_h = labels(Eh, Wh, cost)
    Xh = features(G, ho).cpu().numpy()
    rmax_l, fallbacks = model.predict_rmax(G, ho)
    rmax_l = rmax_l.cpu().numpy()
    rstar = cost["rmax_star"]
    # modelled cost on the held-out sweep (nearest grid point of the prediction)
    pick = np.abs(np.log(rmax_l / rstar)[:, None] - np.log(MULTS)[None, :]).argmin(1)
    i_star = np.abs(np.log(MULTS)).argmin()
    mod_learned = cost_h[np.arange(len(ho)), pick]
    mod_fixed = cost_h[:, i_star]
    # the best single multiplier for all sources (what a global retuning of
    # eqn:rmax would reach, with no per-source model)
    i_glob = int(np.argmin(cost_h.sum(0)))
    timed = ho[:args.timed]
    log("timing single queries")
    t_fixed = time_queries(G, timed)
    t_learn = time_queries(G, timed, rmax=rmax_l[:args.timed])
    t_glob = time_queries(G, timed, rmax=np.full(len(timed), rstar * MULTS[i_glob]))
    log("timing batched queries")
    qps_fixed = time_batched(G, ho)
    qps_learn = time_batched(G, ho, rmax=rmax_l)
    t_inf0 = time.perf_counter()
    model.predict_rmax(G, ho)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t_inf0

    def summary(t):
        return dict(mean=float(t.mean()), p50=float(np.percentile(t, 50)),
                    p95=float(np.percentile(t, 95)))

    rep = dict(workload=args.workload, n=g.n, m=g.m, train=len(tr), heldout=len(ho),
               grid=MULTS.tolist(), unit_costs=cost,
               label_mult_histogram=np.bincount(np.argmin(np.abs(y[:, None] - np.log(MULTS)), 1),
                                                minlength=len(MULTS)).tolist(),
               label_std=float(y.std()),
               train_mse=model.mse(X, y), heldout_mse=model.mse(Xh, yh),
               heldout_mse_fixed_rule=float(np.mean(yh ** 2)),
               heldout_mse_best_constant=float(np.mean((yh - y.mean()) ** 2)),
               fallbacks=fallbacks,
               modelled_cost_ms=dict(fixed_mean=float(mod_fixed.mean()),
                                     learned_mean=float(mod_learned.mean()),
                                     best_global_mult=float(MULTS[i_glob]),
                                     best_global_mean=float(cost_h[:, i_glob].mean()),
                                     per_source_best_mean=float(cost_h.min(1).mean())),
               measured_single_query_ms=dict(sources=int(len(timed)), fixed=summary(t_fixed),
                                             learned=summary(t_learn),
                                             best_global_mult=summary(t_glob)),
               batched_queries_per_s=dict(fixed=qps_fixed, learned=qps_learn),
               sweep_seconds=t_sweep, train_seconds=t_train,
               inference_us_per_source=t_inf / len(ho) * 1e6)
    print(json.dumps(rep), flush=True)
    return rep


if __name__ == "__main__":
    main()
