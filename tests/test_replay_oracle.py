"""Pins of the oracle's frontier replay (Algorithm 1 with the frontiers of
another run given; CPU only).

Replaying the oracle's own frontiers rebuilds its push bit for bit; wrong
frontiers are reported (a listed node below its threshold, a node left over
it); any replayed sequence keeps eqn:layerppr against the dense solve; and
replaying the frontiers of an FP32 push that sums in another order, on a
case where a residue sits exactly on its threshold so that the two runs
push different nodes, reconciles the two states element by element."""
import numpy as np
import pytest

import oracle
import synth
from oracle import exact

ALPHA = 0.2
TAU = 1e-5


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def g10():
    return synth.rmat_graph(10, seed=3, cache=False)


@pytest.mark.parametrize("s,rmax", [(0, 3.754e-5), (17, 1e-3), (999, 1e-6)])
def test_replay_of_own_frontiers_is_bit_exact(g1k, s, rmax):
    ref = oracle.push(g1k, s, ALPHA, rmax, log_frontiers=True)
    rep = oracle.push_replay(g1k, s, ALPHA, rmax, ref["frontiers"])
    assert np.array_equal(rep["r"], ref["r"]) and np.array_equal(rep["q"], ref["q"])
    # every listed node passed the test, none was left over its threshold,
    # and the closest call is the oracle's own margin
    assert rep["max_listed_shortfall"] < 0 and rep["max_unlisted_excess"] <= 0
    assert min(-rep["max_listed_shortfall"], -rep["max_unlisted_excess"]) == \
        pytest.approx(ref["min_margin"], rel=1e-12)


def test_wrong_frontiers_are_reported(g1k):
    rmax = 1e-4
    ref = oracle.push(g1k, 0, ALPHA, rmax, log_frontiers=True)
    fr = [f.copy() for f in ref["frontiers"]]
    # the source left out of round 0: it stays far over its threshold
    rep = oracle.push_replay(g1k, 0, ALPHA, rmax, [fr[0][:0]] + fr[1:])
    assert rep["max_unlisted_excess"] > 1.0
    # a node with no residue listed in the second push round: short by its whole threshold
    idle = int(np.setdiff1d(np.arange(g1k.n), fr[1])[0])
    extra = np.sort(np.concatenate([fr[1], [idle]]))
    rep = oracle.push_replay(g1k, 0, ALPHA, rmax, [fr[0], extra] + fr[2:])
    assert rep["max_listed_shortfall"] == pytest.approx(1.0)
    # the last round left out: its nodes end over their thresholds
    rep = oracle.push_replay(g1k, 0, ALPHA, rmax, fr[:-1])
    assert rep["max_unlisted_excess"] > 0
    with pytest.raises(ValueError):
        oracle.push_replay(g1k, 0, ALPHA, rmax, [fr[0], fr[1][::-1]] + fr[2:])


def test_any_replayed_sequence_keeps_the_invariant(g1k):
    # eqn:layerppr holds for every sequence of pushes: hold back half of each
    # round's frontier by one round (pushing late, or pushing a node whose
    # residue has grown) and compare with the dense solve
    Pi = exact.dense_ppr(g1k, ALPHA)
    rmax = 1e-4
    ref = oracle.push(g1k, 0, ALPHA, rmax, log_frontiers=True)
    late = []
    held = np.zeros(0, np.int64)
    for f in ref["frontiers"]:
        now = np.union1d(f[::2], held)
        held = f[1::2]
        late.append(now)
    late.append(held)
    rep = oracle.push_replay(g1k, 0, ALPHA, rmax, late)
    np.testing.assert_allclose(rep["q"] + rep["r"] @ Pi, Pi[0], atol=1e-12)
    assert rep["q"].sum() + rep["r"].sum() == pytest.approx(1.0, abs=1e-12)


def _push_fp32_other_order(g, s, alpha, rmax):
    """A synchronous push in FP32 (the residue promoted to FP64 for the test,
    as the device does) that adds each round's increments in reverse edge
    order: a model of a correct FP32 run whose rounding differs."""
    rp = np.asarray(g.rowptr, np.int64)
    ci = np.asarray(g.colidx, np.int64)
    deg = np.diff(rp)
    thr = rmax * deg.astype(np.float64)
    r = np.zeros(g.n, np.float32)
    q = np.zeros(g.n, np.float32)
    r[s] = 1.0
    a32, b32 = np.float32(alpha), np.float32(1.0 - alpha)
    frontiers = []
    while True:
        F = np.flatnonzero(r.astype(np.float64) > thr)
        if F.size == 0:
            return r, q, frontiers
        frontiers.append(F)
        x = r[F].copy()
        r[F] = 0
        q[F] += a32 * x
        d = deg[F]
        inc = (b32 * x) / d.astype(np.float32)
        edges = np.repeat(rp[F] - (np.cumsum(d) - d), d) + np.arange(int(d.sum()))
        np.add.at(r, ci[edges][::-1], np.repeat(inc, d)[::-1])


def test_replay_reconciles_a_push_with_other_rounding(g10):
    # r_max chosen so that an out-neighbour u of s holds exactly its
    # threshold after round 0 in FP64: the FP32 run rounds (1-alpha)/d(s) to
    # one side of it and pushes a different set of nodes
    deg = g10.degrees()
    s = 0
    flips = 0
    for u in g10.colidx[g10.rowptr[s]:g10.rowptr[s + 1]][:3]:
        rmax = ((1.0 - ALPHA) / deg[s]) / deg[u]
        free = oracle.push(g10, s, ALPHA, rmax, log_frontiers=True)
        r32, q32, fr = _push_fp32_other_order(g10, s, ALPHA, rmax)
        if len(fr) == free["rounds"] and all(np.array_equal(a, b)
                                              for a, b in zip(fr, free["frontiers"])):
            continue
        flips += 1
        # free running, the states are far apart ...
        assert np.abs(free["q"] - q32).sum() > 1e-4
        # ... replayed in FP64, every listed node passed within rounding, none
        # was left over, and the states agree element by element
        rep = oracle.push_replay(g10, s, ALPHA, rmax, fr)
        assert rep["max_listed_shortfall"] <= TAU and rep["max_unlisted_excess"] <= TAU
        np.testing.assert_allclose(q32, rep["q"], rtol=TAU, atol=1e-12)
        np.testing.assert_allclose(r32, rep["r"], rtol=TAU, atol=1e-12)
    assert flips >= 1
