"""CPU oracle for FORA whole-graph SSPPR (Algorithms 1 and 2 of the paper,
r_max by eqn:rmax), plus exact PPR references and the MLP reference.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does. It is
independent of the HIP implementation (no shared code, constants or helpers);
both take their inputs from ``synth``.

The arithmetic lives in ``fora_oracle.c`` (plain single-threaded C, FP64);
this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fora_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (single-threaded, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    lib.oracle_philox4x32_10.argtypes = [P, P, P]
    lib.oracle_philox_many.argtypes = [i64, P, P, P]
    lib.oracle_validate.argtypes = [i32, i64, P, P]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_constants.argtypes = [i64, f64, f64, f64, f64, f64, P]
    lib.oracle_push.argtypes = [i32, P, P, i32, f64, f64, P, P, i32, P, P, P, i64, P]
    lib.oracle_push.restype = i32
    lib.oracle_push_continue.argtypes = [i32, P, P, f64, f64, P, P, i32, P, P, P, i64, P]
    lib.oracle_push_continue.restype = i32
    lib.oracle_plan.argtypes = [i32, P, f64, P, P, P]
    lib.oracle_plan.restype = i64
    lib.oracle_walks.argtypes = [i32, P, P, u32, u32, u32, i64, P, P, P, i32, P, P, P, P]
    lib.oracle_push_balanced.argtypes = [i32, P, P, i32, f64, f64, f64, f64, P, P, i32, P, P,
                                         P, i64, P, P, P]
    lib.oracle_push_balanced.restype = i32
    lib.oracle_push_replay.argtypes = [i32, P, P, f64, f64, P, P, i32, P, P, P]
    lib.oracle_push_replay.restype = i32
    lib.oracle_topk.argtypes = [i32, P, i32, P, P]
    lib.oracle_topk.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    rp = np.ascontiguousarray(g.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.colidx, dtype=np.int32)
    return rp, ci


# --------------------------------------------------------------------------
def philox(ctrs: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 blocks for an array of 4-word counters."""
    lib = _load()
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(c)
    lib.oracle_philox_many(c.shape[0], _p(c), _p(k), _p(out))
    return out


def validate(g) -> int:
    rp, ci = _csr(g)
    return _load().oracle_validate(rp.shape[0] - 1, ci.shape[0], _p(rp), _p(ci))


def constants(m: int, alpha: float, eps: float, delta: float, pf: float,
              rmax: float | None = None) -> dict:
    out = np.zeros(5, np.float64)
    _load().oracle_constants(m, alpha, eps, delta, pf,
                             0.0 if rmax is None else float(rmax), _p(out))
    return dict(c=out[0], L=out[1], omega_unit=out[2], rmax=out[3],
                t_alpha=int(out[4]))


def push(g, s: int, alpha: float, rmax: float, max_rounds: int = 100000,
         log_frontiers: bool = False, frontier_cap: int | None = None) -> dict:
    """Synchronous Forward Push; returns r, q (FP64) and per-round data."""
    lib = _load()
    rp, ci = _csr(g)
    n = rp.shape[0] - 1
    r = np.zeros(n, np.float64)
    q = np.zeros(n, np.float64)
    sizes = np.zeros(max_rounds, np.int32)
    ops = np.zeros(1, np.int64)
    margin = np.zeros(1, np.float64)
    cap = 0
    flog = None
    if log_frontiers:
        cap = frontier_cap if frontier_cap is not None else 64 * n
        flog = np.zeros(cap, np.int32)
    rounds = lib.oracle_push(n, _p(rp), _p(ci), int(s), alpha, rmax, _p(r), _p(q),
                             max_rounds, _p(sizes), _p(ops), _p(flog), cap,
                             _p(margin))
    if rounds < 0:
        raise RuntimeError(f"oracle_push failed ({rounds})")
    sizes = sizes[:rounds].copy()
    out = dict(r=r, q=q, rounds=int(rounds), round_sizes=sizes,
               edge_ops=int(ops[0]), min_margin=float(margin[0]))
    if log_frontiers:
        offs = np.concatenate([[0], np.cumsum(sizes)])
        out["frontiers"] = [flog[offs[i]:offs[i + 1]].copy() for i in range(rounds)]
    return out


def push_replay(g, s: int, alpha: float, rmax: float, frontiers, r0=None) -> dict:
    """Algorithm 1 with the frontier of every synchronous round given rather
    than tested, from r = e_s (or r = r0, a source distribution), q = 0.
    Algorithm 1 may push nodes in any order and eqn:layerppr holds for every
    sequence of pushes, so replaying another run's frontiers in FP64 rebuilds
    the state that run should have reached. Each round pushes its listed
    nodes (ascending) exactly as the oracle's synchronous push does.

    Before each round it measures how far the listed nodes are from the push
    test r(v) > r_max d(v) and how far the unlisted ones are over it, both
    relative to the threshold; after the last round, how far any node is
    over it. Returns r and q (FP64), max_listed_shortfall (the largest
    (r_max d(v) - r(v)) / (r_max d(v)) over listed nodes: negative when every
    listed node passes the test) and max_unlisted_excess (the largest
    (r(v) - r_max d(v)) / (r_max d(v)) over unlisted nodes and the final
    state: at most 0 when no node was left over its threshold)."""
    if not rmax > 0.0:
        raise ValueError("rmax must be positive")
    lib = _load()
    rp, ci = _csr(g)
    n = rp.shape[0] - 1
    if r0 is None:
        r = np.zeros(n, np.float64)
        r[int(s)] = 1.0
    else:
        r = np.array(r0, np.float64, copy=True).reshape(n)
    q = np.zeros(n, np.float64)
    frontiers = [np.asarray(F, np.int32).reshape(-1) for F in frontiers]
    sizes = np.array([F.size for F in frontiers], np.int64)
    flat = np.ascontiguousarray(np.concatenate(frontiers) if frontiers else
                                np.zeros(0, np.int32), np.int32)
    out = np.zeros(2, np.float64)
    rc = lib.oracle_push_replay(n, _p(rp), _p(ci), alpha, rmax, _p(r), _p(q), len(frontiers),
                                _p(sizes), _p(flat), _p(out))
    if rc == -1:
        raise ValueError("a frontier must hold distinct node ids in ascending order")
    if rc != 0:
        raise RuntimeError(f"oracle_push_replay failed ({rc})")
    return dict(r=r, q=q, rounds=len(frontiers), max_listed_shortfall=float(out[0]),
                max_unlisted_excess=float(out[1]))


def push_sweep(g, s: int, alpha: float, rmaxes, omega_unit: float,
               max_rounds: int = 100000) -> dict:
    """Algorithm 1 at r_max = rmaxes[0], then continued from the state it
    left at each lower threshold in turn (the loop of Algorithm 1 only needs
    a state, not r = e_s). After threshold i: cumulative edge operations
    E[i] and the walk count Algorithm 2 would then run, W[i] = sum_v
    ceil(r(v) omega_unit); min_margin is the smallest relative distance of a
    tested residue from its threshold over the whole sweep."""
    lib = _load()
    rp, ci = _csr(g)
    n = rp.shape[0] - 1
    r = np.zeros(n, np.float64)
    q = np.zeros(n, np.float64)
    r[int(s)] = 1.0
    sizes = np.zeros(max_rounds, np.int32)
    ops = np.zeros(1, np.int64)
    margin = np.zeros(1, np.float64)
    E, W, total, mmin = [], [], 0, math.inf
    for rm in rmaxes:
        rounds = lib.oracle_push_continue(n, _p(rp), _p(ci), alpha, float(rm), _p(r), _p(q),
                                          max_rounds, _p(sizes), _p(ops), None, 0, _p(margin))
        if rounds < 0:
            raise RuntimeError(f"oracle_push_continue failed ({rounds})")
        total += int(ops[0])
        mmin = min(mmin, float(margin[0]))
        E.append(total)
        W.append(int(np.ceil(r[r > 0] * omega_unit).sum()))
    return dict(E=np.array(E, np.int64), W=np.array(W, np.int64), r=r, q=q, min_margin=mmin)


def plan(r: np.ndarray, omega_unit: float):
    """Walk plan (v, omega_v, w_v) for v ascending with r(v) > 0."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    pv = np.zeros(n, np.int32)
    po = np.zeros(n, np.uint64)
    pw = np.zeros(n, np.float64)
    e = lib.oracle_plan(n, _p(r), omega_unit, _p(pv), _p(po), _p(pw))
    if e < 0:
        raise OverflowError("a per-node walk count does not fit in 32 bits")
    return pv[:e].copy(), po[:e].copy(), pw[:e].copy()


def push_balanced(g, s: int, alpha: float, rmax: float, omega_unit: float, walk_cost: float,
                  max_rounds: int = 100000, log_frontiers: bool = False) -> dict:
    """Algorithm 3's push: synchronous Algorithm 1 that also stops once the
    edge operations done reach the estimated walk cost,
    (1 - alpha * pushed mass) (1 - alpha) omega_unit walk_cost."""
    lib = _load()
    rp, ci = _csr(g)
    n = rp.shape[0] - 1
    r = np.zeros(n, np.float64)
    q = np.zeros(n, np.float64)
    sizes = np.zeros(max_rounds, np.int32)
    ops = np.zeros(1, np.int64)
    margin = np.zeros(1, np.float64)
    bmargin = np.zeros(1, np.float64)
    stopped = np.zeros(1, np.int32)
    cap = 64 * n if log_frontiers else 0
    flog = np.zeros(cap, np.int32) if log_frontiers else None
    rounds = lib.oracle_push_balanced(n, _p(rp), _p(ci), int(s), alpha, rmax, omega_unit,
                                      float(walk_cost), _p(r), _p(q), max_rounds, _p(sizes),
                                      _p(ops), _p(flog), cap, _p(margin), _p(bmargin),
                                      _p(stopped))
    if rounds < 0:
        raise RuntimeError(f"oracle_push_balanced failed ({rounds})")
    sizes = sizes[:rounds].copy()
    out = dict(r=r, q=q, rounds=int(rounds), round_sizes=sizes, edge_ops=int(ops[0]),
               min_margin=float(margin[0]), balance_margin=float(bmargin[0]),
               stopped=bool(stopped[0]))
    if log_frontiers:
        offs = np.concatenate([[0], np.cumsum(sizes)])
        out["frontiers"] = [flog[offs[i]:offs[i + 1]].copy() for i in range(rounds)]
    return out


def walks(g, source: int, seed: int, t_alpha: int, plan_v, plan_omega, plan_w,
          endpoints: bool = False, first_move: bool = False) -> dict:
    """Run every planned walk; endpoint counts, weighted sums and step total.
    first_move: every walk's first step is a forced move (Algorithm 3)."""
    lib = _load()
    rp, ci = _csr(g)
    n = rp.shape[0] - 1
    pv = np.ascontiguousarray(plan_v, dtype=np.int32)
    po = np.ascontiguousarray(plan_omega, dtype=np.uint64)
    pw = np.ascontiguousarray(plan_w, dtype=np.float64)
    cnt = np.zeros(n, np.uint64)
    acc = np.zeros(n, np.float64)
    steps = np.zeros(1, np.uint64)
    W = int(po.sum())
    ends = np.zeros(W, np.int32) if endpoints else None
    lib.oracle_walks(n, _p(rp), _p(ci), source & 0xFFFFFFFF, seed & 0xFFFFFFFF,
                     t_alpha, pv.shape[0], _p(pv), _p(po), _p(pw), int(bool(first_move)),
                     _p(cnt), _p(acc), _p(steps), _p(ends))
    out = dict(cnt=cnt, acc=acc, steps=int(steps[0]), walks=W)
    if endpoints:
        out["endpoints"] = ends
    return out


def topk(pi: np.ndarray, k: int):
    lib = _load()
    pi = np.ascontiguousarray(pi, dtype=np.float64)
    ids = np.zeros(k, np.int32)
    vals = np.zeros(k, np.float64)
    rc = lib.oracle_topk(pi.shape[0], _p(pi), k, _p(ids), _p(vals))
    if rc != 0:
        raise ValueError("bad k")
    return ids, vals


def fora(g, s: int, alpha: float = 0.2, eps: float = 0.5, delta: float | None = None,
         pf: float | None = None, k: int = 500, seed: int = 0,
         rmax: float | None = None, log_frontiers: bool = False, prune: bool = False,
         walk_cost: float | None = None, walk_key=None) -> dict:
    """Whole-graph FORA (Algorithm 2) followed by top-k selection.

    prune: Algorithm 3's zero-hop pruning (section 4.1): pi_hat starts at
    q + alpha r, and from each v with residue ceil(r'(v) omega_unit) walks
    with r' = (1 - alpha) r start at a random out-neighbour of v, each adding
    r'(v) / omega_v at its end point.
    walk_cost: Algorithm 3's balance rule (section 4.2), the cost of one walk
    in edge-operation units (None: plain Algorithm 1).
    walk_key: (key0, key1) of the walks instead of (s, seed): the walks of an
    index shared by all sources (FORA+, section 3.3); walk j from v is then
    the j-th pre-computed walk of v whoever the source is."""
    n = g.n
    delta = 1.0 / n if delta is None else delta
    pf = 1.0 / n if pf is None else pf
    if validate(g) != 0:
        raise ValueError("invalid graph")
    c = constants(g.m, alpha, eps, delta, pf, rmax)
    if walk_cost is None:
        ps = push(g, s, alpha, c["rmax"], log_frontiers=log_frontiers)
    else:
        ps = push_balanced(g, s, alpha, c["rmax"], c["omega_unit"], walk_cost,
                           log_frontiers=log_frontiers)
    r_walk = (1.0 - alpha) * ps["r"] if prune else ps["r"]
    pv, po, pw = plan(r_walk, c["omega_unit"])
    k0, k1 = (s, seed) if walk_key is None else walk_key
    wk = walks(g, k0, k1, c["t_alpha"], pv, po, pw, first_move=prune)
    pi = ps["q"] + wk["acc"] + (alpha * ps["r"] if prune else 0.0)
    ids, vals = topk(pi, min(k, n))
    out = dict(consts=c, plan=(pv, po, pw), pi=pi, topk_ids=ids, topk_vals=vals,
               r_sum=float(ps["r"].sum()))
    out.update(ps)
    out.update(wk)
    return out

DIST_KEY0 = 0xFFFFFFFF  # first Philox key word of walks for a source distribution


def fora_dist(g, sigma, alpha: float = 0.2, eps: float = 0.5, delta: float | None = None,
              pf: float | None = None, k: int = 500, seed: int = 0,
              rmax: float | None = None, log_frontiers: bool = False) -> dict:
    """FORA for a source distribution sigma (section 6.2, the paper's extension to source
    distributions): Algorithm 1 starts from r = sigma, q = 0 instead of
    r = e_s, which keeps the invariant pi(sigma, t) = q(t) + sum_v r(v)
    pi(v, t); Algorithm 2 and the selection are unchanged. Global PageRank is
    sigma = (1/n, ..., 1/n). Walks are keyed by (DIST_KEY0, seed)."""
    n = g.n
    delta = 1.0 / n if delta is None else delta
    pf = 1.0 / n if pf is None else pf
    sigma = np.asarray(sigma, np.float64)
    if sigma.shape != (n,) or not np.all(np.isfinite(sigma)) or np.any(sigma < 0):
        raise ValueError("sigma must be n finite non-negative values")
    if validate(g) != 0:
        raise ValueError("invalid graph")
    c = constants(g.m, alpha, eps, delta, pf, rmax)
    lib = _load()
    rp, ci = _csr(g)
    r = sigma.copy()
    q = np.zeros(n, np.float64)
    max_rounds = 100000
    sizes = np.zeros(max_rounds, np.int32)
    ops = np.zeros(1, np.int64)
    margin = np.zeros(1, np.float64)
    cap = 64 * n if log_frontiers else 0
    flog = np.zeros(cap, np.int32) if log_frontiers else None
    rounds = lib.oracle_push_continue(n, _p(rp), _p(ci), alpha, c["rmax"], _p(r), _p(q),
                                      max_rounds, _p(sizes), _p(ops), _p(flog), cap, _p(margin))
    if rounds < 0:
        raise RuntimeError(f"oracle_push_continue failed ({rounds})")
    sizes = sizes[:rounds].copy()
    pv, po, pw = plan(r, c["omega_unit"])
    wk = walks(g, DIST_KEY0, seed, c["t_alpha"], pv, po, pw)
    pi = q + wk["acc"]
    ids, vals = topk(pi, min(k, n))
    out = dict(consts=c, plan=(pv, po, pw), pi=pi, topk_ids=ids, topk_vals=vals, r=r, q=q,
               rounds=int(rounds), round_sizes=sizes, edge_ops=int(ops[0]),
               min_margin=float(margin[0]), r_sum=float(r.sum()))
    if log_frontiers:
        offs = np.concatenate([[0], np.cumsum(sizes)])
        out["frontiers"] = [flog[offs[i]:offs[i + 1]].copy() for i in range(rounds)]
    out.update(wk)
    return out


def topk_deltas(n: int, k: int):
    """Algorithm 5's thresholds: delta = 1/k, 1/(2k), ... while above 1/n,
    then 1/n (the last iteration returns whatever it finds)."""
    out = []
    d = 1.0 / k
    while d > 1.0 / n:
        out.append(d)
        d /= 2.0
    out.append(1.0 / n)
    return out


def fora_topk(g, s: int, k: int, alpha: float = 0.2, eps: float = 0.5, pf: float | None = None,
              seed: int = 0, prune: bool = False) -> dict:
    """Top-k FORA (Algorithm 5): for delta = 1/k, 1/(2k), ..., 1/n run
    Algorithm 2 with eps' = eps / 2, p_f' = p_f / (n log2(n / k)) and r_max by
    eqn:rmax for those parameters (iteration i uses Philox seed seed + i);
    stop at the first iteration whose k-th largest estimate (rounded to FP32,
    the precision the result is returned in) is at least (1 + eps) delta."""
    n = g.n
    pf = 1.0 / n if pf is None else pf
    pf_it = pf / (n * max(math.log2(n / k), 1.0))
    trace = []
    out = None
    deltas = topk_deltas(n, k)
    for i, d in enumerate(deltas):
        out = fora(g, s, alpha=alpha, eps=eps / 2, delta=d, pf=pf_it, k=k, seed=seed + i,
                   prune=prune)
        kth = float(np.float32(out["topk_vals"][k - 1]))
        trace.append(dict(delta=d, kth=kth, bound=(1 + eps) * d,
                          omega_unit=out["consts"]["omega_unit"]))
        if kth >= (1 + eps) * d or i == len(deltas) - 1:
            break
    out = dict(out)
    out.update(iterations=len(trace), delta=trace[-1]["delta"], trace=trace, pf_iter=pf_it)
    return out


def build_index(g, alpha: float, walks_per_degree: float, key) -> dict:
    """FORA+'s walk-destination index (section 3.3, eqn:index-rwnum): for
    every node v, omega_max(v) = ceil(d(v) walks_per_degree) walks (with
    walks_per_degree = r_max omega_unit) keyed by (key0, key1) and walk
    index j; their end points in (v, j) order, and the offsets."""
    n = g.n
    deg = g.degrees().astype(np.float64)
    om = np.ceil(deg * walks_per_degree).astype(np.uint64)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum(om)
    t_alpha = int(math.floor(alpha * 2.0**32))
    pv = np.arange(n, dtype=np.int32)
    wk = walks(g, key[0], key[1], t_alpha, pv, om, np.ones(n), endpoints=True)
    return dict(off=off, dest=wk["endpoints"], omega_max=om)
