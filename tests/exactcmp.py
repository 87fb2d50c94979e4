"""Element-wise comparison of the device's push and walks with the oracle.

The device's push is order-independent (fixed-point residues summed as
integers), so the same query gives the same frontiers, residues and
reserves in every run and in every batch. Against the FP64 oracle it may
still differ where a residue lies within rounding of its threshold: then
the two runs push different nodes (Algorithm 1 allows any order; the
rounding decides). The frontier replay settles every such case: the
oracle applies the device's own frontiers in FP64 and reports how close
each listed node was to passing the test and each unlisted one to failing
it; within the tolerance both runs are correct, and r and q must then agree
element by element with the replayed state.

The walk phase is a function of the residues alone (omega_v and the weights
come from r, every walk is keyed by (source, seed, start node, walk index,
step)), so the oracle's plan and walks on the device's own residues must
reproduce the device's end-point counts and move count exactly.
"""
import numpy as np

import oracle

TAU = 1e-5  # relative tolerance of the push test and of r, q (FP32 reserve)
ATOL = 1e-12


def close(g, o, rtol=TAU, atol=ATOL):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return np.abs(g - o) <= rtol * np.abs(o) + atol


def check_push(g, s, alpha, rmax, frontiers, r_dev, q_dev, r0=None):
    """Replays the device's frontiers in the oracle; asserts the push test
    held for every listed node and no unlisted node was over its threshold
    (both within TAU), and r and q element-wise. Returns the replay."""
    rep = oracle.push_replay(g, s, alpha, rmax, frontiers, r0=r0)
    assert rep["max_listed_shortfall"] <= TAU, rep["max_listed_shortfall"]
    assert rep["max_unlisted_excess"] <= TAU, rep["max_unlisted_excess"]
    r_dev = np.asarray(r_dev, np.float64)
    q_dev = np.asarray(q_dev, np.float64)
    bad_r = ~close(r_dev, rep["r"])
    bad_q = ~close(q_dev, rep["q"])
    assert not bad_r.any(), (int(bad_r.sum()), np.flatnonzero(bad_r)[:5])
    assert not bad_q.any(), (int(bad_q.sum()), np.flatnonzero(bad_q)[:5])
    return rep


def oracle_walks_on(g, r_dev, omega_unit, key0, key1, t_alpha, scale=1.0, first_move=False,
                    workers=1):
    """The oracle's plan and walks on the device's residues (FP64 copies of
    the fixed-point values, scaled by `scale` for Algorithm 3). With
    workers > 1 the plan is cut into pieces walked in forked processes: walks
    are keyed by (start node, walk index), so the integer counts and step
    totals of the pieces add up to those of the whole plan."""
    r = np.asarray(r_dev, np.float64)
    pv, po, pw = oracle.plan(scale * r if scale != 1.0 else r, omega_unit)
    if workers <= 1 or len(pv) < 2 * workers:
        w = oracle.walks(g, key0, key1, t_alpha, pv, po, pw, first_move=first_move)
        return dict(cnt=w["cnt"], acc=w["acc"], steps=w["steps"], walks=int(po.sum()))
    import multiprocessing as mp
    # pieces of about equal walk counts
    cum = np.cumsum(po.astype(np.float64))
    cuts = np.searchsorted(cum, np.linspace(0, cum[-1], 4 * workers + 1)[1:-1])
    bounds = np.unique(np.concatenate([[0], cuts, [len(pv)]]))
    jobs = [(g, key0, key1, t_alpha, pv[a:b], po[a:b], pw[a:b], first_move)
            for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_walk_piece, jobs)
    cnt = np.zeros(g.n, np.uint64)
    acc = np.zeros(g.n, np.float64)
    steps = 0
    for c, a, st in parts:
        cnt += c
        acc += a
        steps += st
    return dict(cnt=cnt, acc=acc, steps=steps, walks=int(po.sum()))


def _walk_piece(job):
    g, k0, k1, ta, pv, po, pw, fm = job
    w = oracle.walks(g, k0, k1, ta, pv, po, pw, first_move=fm)
    return w["cnt"], w["acc"], int(w["steps"])


def check_walks(ref, cnt_dev, steps_dev, acc_fx_dev=None):
    """Device end-point counts and moves equal the oracle's on the same plan
    (steps_dev None: moves not compared, for walks read from an index);
    fixed-point weights within the rounding of round(w 2^62) per walk."""
    cnt = np.asarray(cnt_dev).view(np.uint64) if np.asarray(cnt_dev).dtype != np.uint64 \
        else np.asarray(cnt_dev)
    assert np.array_equal(cnt, ref["cnt"])
    if steps_dev is not None:
        assert int(steps_dev) == int(ref["steps"])
    if acc_fx_dev is not None:
        acc = np.asarray(acc_fx_dev).view(np.uint64).astype(np.float64) / 2.0**62
        tol = ref["cnt"] * 2.0**-62 + 1e-15 * ref["acc"]
        assert np.all(np.abs(acc - ref["acc"]) <= tol)


def row_of(views, i):
    """Query i's row of the workspace views as numpy arrays."""
    return {k: t[i].cpu().numpy() for k, t in views.items()}


def check_query(g, G, s, alpha, rmax, row, stats, key0=None, key1=0, workers=1, scale=1.0,
                first_move=False, steps=True):
    """One query of a finished call against the oracle, element by element.

    row: the query's workspace row (row_of), from a call that counted walk
    end points (FORA_WALK_COUNTS); stats: its fora_stats. The device's push
    is run again on its own with its frontiers logged; it must equal the
    call's row bit for bit (the push does not depend on the batch). The
    oracle replays those frontiers (check_push), then walks the plan of the
    device's residues: counts and moves must be equal, weights within the
    fixed-point rounding. Returns the replay and the walks."""
    from paper_1908_10583_amd import fora
    p = fora.fora_push_only(G, int(s), alpha, rmax, log_frontiers=True)
    assert np.array_equal(p["r_fx"].cpu().numpy(), row["residue_fx"])
    assert np.array_equal(p["q"].cpu().numpy(), row["reserve"])
    assert p["stats"]["rounds"] == stats["rounds"]
    rep = check_push(g, s, alpha, rmax, p["frontiers"], row["residue"], row["reserve"])
    del p
    t_alpha = int(np.floor(np.ldexp(alpha, 32)))
    k0 = int(s) if key0 is None else key0
    ref = oracle_walks_on(g, row["residue"], stats["omega_unit"], k0, key1, t_alpha,
                          scale=scale, first_move=first_move, workers=workers)
    assert ref["walks"] == stats["walks"]
    check_walks(ref, row["walk_count"], stats["steps"] if steps else None,
                row["walk_weight_fx"])
    return rep, ref


def check_topk_iterations(g, G, s, alpha, k, seed, iters, delta, ids, vals, eps=0.5,
                          workers=1):
    """Top-k FORA (Algorithm 5) of source s took `iters` iterations and ended
    at `delta` with result (ids, vals): reruns each iteration as a plain query
    (eps / 2, p_f / (n log2(n / k)), that iteration's delta, seed + iteration)
    and checks it against the oracle (check_query), the stopping rule on its
    k-th estimate, and that the result is the last iteration's bit for bit."""
    from paper_1908_10583_amd import fora
    n = g.n
    pf_it = (1.0 / n) / (n * max(np.log2(n / k), 1.0))
    deltas = oracle.topk_deltas(n, k)
    assert delta == deltas[iters - 1]
    ws = fora.workspace(G, 1)
    for it in range(iters):
        one = fora.fora_ssppr(G, s, alpha, eps / 2, deltas[it], pf_it, k, seed=seed + it, ws=ws,
                              stats=True, flags=fora.FORA_WALK_COUNTS)
        row = row_of(fora.fora_workspace_views(G, 1, ws), 0)
        check_query(g, G, s, alpha, one.stats["rmax"], row, one.stats, key1=seed + it,
                    workers=workers)
        kth = float(one.vals[k - 1].cpu())
        stop = kth >= (1 + eps) * deltas[it] or it == len(deltas) - 1
        assert stop == (it == iters - 1), (it, kth, deltas[it])
    assert np.array_equal(one.ids.cpu().numpy(), ids[:k])
    assert np.array_equal(one.vals.cpu().numpy(), vals[:k])
