"""Pins of the oracle's Algorithm 3 parts (section 4): zero-hop pruning and
the push/walk balance rule. CPU only.

Pruning is pinned by the decomposition pi = pi_0 + pi_1 of section 4.1: a
walk that must move first ends at t with probability
(pi(v,t) - alpha [v = t]) / (1 - alpha) (checked against the dense solve),
its length minus one is geometric, the estimator stays unbiased and keeps the
eps guarantee. The balance rule is pinned by its two limits (a zero walk cost
pushes nothing, an unbounded one is plain Algorithm 1), by eqn:layerppr at
the state where it stops, and by the stop condition restated with the
reserves (pushed mass = sum q / alpha)."""
import math

import numpy as np
import pytest
import scipy.stats as st

import oracle
import synth
from oracle import exact
from synth.graphs import Graph

ALPHA = 0.2


def _chi2_pvalue(obs, expected):
    obs = np.asarray(obs, np.float64)
    expected = np.asarray(expected, np.float64)
    keep = expected >= 5
    o, e = obs[keep], expected[keep]
    if (~keep).any():
        o = np.append(o, obs[~keep].sum())
        e = np.append(e, expected[~keep].sum())
    e = e * (o.sum() / e.sum())
    return st.chisquare(o, e).pvalue


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def pi1k(g1k):
    return exact.dense_ppr(g1k, ALPHA)


def _walks(g, v, omega, first_move, seed=0):
    t_alpha = oracle.constants(g.m, ALPHA, 0.5, 0.01, 0.01)["t_alpha"]
    return oracle.walks(g, 0, seed, t_alpha, np.array([v], np.int32),
                        np.array([omega], np.uint64), np.array([1.0 / omega]),
                        endpoints=True, first_move=first_move)


def test_forced_first_move_ends_by_pi_one(g1k, pi1k):
    v, W = 3, 400000
    res = _walks(g1k, v, W, True)
    hist = np.bincount(res["endpoints"], minlength=g1k.n)
    pi1 = pi1k[v].copy()
    pi1[v] -= ALPHA  # pi_0(v, t) = alpha [v = t]
    assert pi1.min() >= -1e-12
    assert _chi2_pvalue(hist, pi1 / (1 - ALPHA) * W) > 1e-6


def test_forced_first_move_lengths():
    # directed cycle: the end point is the walk length mod L; every length is
    # at least one and length - 1 is geometric with stop probability alpha
    L = 64
    g = Graph(np.arange(L + 1, dtype=np.int32), ((np.arange(L) + 1) % L).astype(np.int32))
    W = 200000
    res = _walks(g, 0, W, True)
    hist = np.bincount(res["endpoints"], minlength=L)
    # length l >= 1 ends at l mod L; length L wraps to 0
    p = np.zeros(L)
    for lv in range(1, 40 * L):
        p[lv % L] += ALPHA * (1 - ALPHA) ** (lv - 1)
    assert _chi2_pvalue(hist, p * W) > 1e-6
    assert res["steps"] >= W
    mean_len = res["steps"] / W
    assert abs(mean_len - 1 / ALPHA) < 5 * math.sqrt((1 - ALPHA) / ALPHA**2 / W)
    # the step-0 block picks the move, so the first end point differs from
    # the unforced walk's only where that walk stopped at once
    plain = _walks(g, 0, W, False)
    assert np.count_nonzero(plain["endpoints"] == 0) > 0.15 * W
    assert np.count_nonzero(res["endpoints"] == 0) < 0.01 * W


@pytest.fixture(scope="module")
def repeated_pruned(g1k):
    R = 300
    return np.stack([oracle.fora(g1k, 0, k=50, seed=s, prune=True)["pi"] for s in range(R)])


def test_pruned_estimator_is_unbiased(repeated_pruned, pi1k):
    R = repeated_pruned.shape[0]
    mean = repeated_pruned.mean(0)
    sd = repeated_pruned.std(0, ddof=1)
    mask = (pi1k[0] >= 1e-3) & (sd > 0)
    z = (mean[mask] - pi1k[0][mask]) / (sd[mask] / math.sqrt(R))
    assert np.max(np.abs(z)) < 5.5
    assert np.abs(mean - pi1k[0]).sum() < 0.01


def test_pruned_estimator_keeps_the_guarantee(repeated_pruned, pi1k):
    R = repeated_pruned.shape[0]
    pi = pi1k[0]
    mask = pi >= 1e-3
    fails = (np.abs(repeated_pruned[:, mask] - pi[mask]) > 0.5 * pi[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1e-3).ppf(1 - 1e-6)


def test_pruning_runs_fewer_walks(g1k):
    plain = oracle.fora(g1k, 0, k=50, seed=1)
    pruned = oracle.fora(g1k, 0, k=50, seed=1, prune=True)
    assert pruned["rounds"] == plain["rounds"]
    W, Wp = plain["walks"], pruned["walks"]
    entries = len(plain["plan"][0])
    # sum ceil((1-alpha) r omega) lies within one walk per node of (1-alpha) W
    assert abs(Wp - (1 - ALPHA) * W) <= entries
    assert pruned["pi"].sum() == pytest.approx(1.0, abs=1e-12)


def test_pruned_monte_carlo_case(g1k):
    # no push (r_max >= 1/d(s)): pi_hat(s) gets alpha at once and
    # ceil((1-alpha) omega_unit) walks leave s through a random neighbour
    out = oracle.fora(g1k, 0, k=50, seed=0, rmax=1.0, prune=True)
    assert out["rounds"] == 0
    pv, po, pw = out["plan"]
    assert list(pv) == [0]
    assert int(po[0]) == math.ceil((1 - ALPHA) * out["consts"]["omega_unit"])
    assert out["pi"][0] >= ALPHA


def test_pruned_query_walks_move_at_least_once(g1k):
    # with zero-hop walks pruned every walk of the query makes a forced first
    # move and then a geometric number of further moves: 1 / alpha moves per
    # walk on average (variance (1 - alpha) / alpha^2), against (1 - alpha) /
    # alpha without the forced move
    out = oracle.fora(g1k, 0, k=50, seed=4, prune=True)
    W = out["walks"]
    assert W > 10000
    mean = out["steps"] / W
    assert abs(mean - 1 / ALPHA) < 5 * math.sqrt((1 - ALPHA) / ALPHA**2 / W)


# ---------------------------------------------------------------- balance rule
def test_balance_limits(g1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    plain = oracle.push(g1k, 0, ALPHA, c["rmax"])
    none = oracle.push_balanced(g1k, 0, ALPHA, c["rmax"], c["omega_unit"], 0.0)
    assert none["rounds"] == 0 and none["stopped"] and none["r"][0] == 1.0
    full = oracle.push_balanced(g1k, 0, ALPHA, c["rmax"], c["omega_unit"], 1e30)
    assert not full["stopped"] and full["rounds"] == plain["rounds"]
    np.testing.assert_array_equal(full["r"], plain["r"])
    np.testing.assert_array_equal(full["q"], plain["q"])


def test_balance_stops_where_push_cost_meets_walk_cost(g1k, pi1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    rmax = c["rmax"] / 50  # deep threshold: the balance rule ends the push
    prev_rounds = -1
    for wc in (0.01, 0.05, 0.2, 1.0, 4.0):
        res = oracle.push_balanced(g1k, 0, ALPHA, rmax, c["omega_unit"], wc)
        assert res["stopped"]
        assert res["rounds"] >= prev_rounds
        prev_rounds = res["rounds"]
        r, q = res["r"], res["q"]
        # eqn:layerppr and mass hold wherever the push stops
        np.testing.assert_allclose(q + r @ pi1k, pi1k[0], atol=1e-12)
        assert q.sum() + r.sum() == pytest.approx(1.0, abs=1e-12)
        # the stop condition, with the pushed mass read off the reserves
        r_sum = 1.0 - q.sum()
        est = r_sum * (1 - ALPHA) * c["omega_unit"] * wc
        assert res["edge_ops"] >= est * (1 - 1e-9)
        # and the boundary before did not meet it: the state after one round
        # fewer (plain Algorithm 1 cut after rounds - 1 rounds)
        if res["rounds"] > 0:
            qp, ops = _plain_rounds(g1k, rmax, res["rounds"] - 1)
            est_prev = (1.0 - qp.sum()) * (1 - ALPHA) * c["omega_unit"] * wc
            assert ops < est_prev * (1 + 1e-9)
    assert prev_rounds > 0


def _plain_rounds(g, rmax, rounds):
    """Reserves and edge operations after exactly `rounds` synchronous rounds
    (the C loop stops with its state in place when max_rounds is reached)."""
    import ctypes
    lib = oracle._load()
    n = g.n
    r = np.zeros(n)
    q = np.zeros(n)
    sizes = np.zeros(max(rounds, 1), np.int32)
    ops = np.zeros(1, np.int64)
    rp = np.ascontiguousarray(g.rowptr, np.int32)
    ci = np.ascontiguousarray(g.colidx, np.int32)
    P = lambda a: ctypes.c_void_p(a.ctypes.data)
    lib.oracle_push(n, P(rp), P(ci), 0, ALPHA, rmax, P(r), P(q), rounds, P(sizes), P(ops),
                    None, 0, None)
    return q, int(ops[0])


def test_fora_with_both_parts_keeps_the_guarantee(g1k, pi1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    R = 60
    est = np.stack([oracle.fora(g1k, 0, k=50, seed=s, prune=True, walk_cost=1.0,
                                rmax=c["rmax"] / 20)["pi"] for s in range(R)])
    pi = pi1k[0]
    mask = pi >= 1e-3
    fails = (np.abs(est[:, mask] - pi[mask]) > 0.5 * pi[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1e-3).ppf(1 - 1e-6)
    assert np.abs(est.mean(0) - pi).sum() < 0.02
