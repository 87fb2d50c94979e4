"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here compares the oracle with something other than itself:
hand-worked fixtures, closed forms, the exact PPR from a dense solve,
invariants the paper states, distributions the random-walk definition fixes,
and library routines (sort). No GPU is needed.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats as st

import oracle
import synth
from oracle import exact
from synth.graphs import Graph

from conftest import GOLDEN

ALPHA = 0.2


def _graph(d):
    return Graph(np.array(d["rowptr"], np.int32), np.array(d["colidx"], np.int32))


def _chi2_pvalue(obs, expected):
    """Chi-square goodness of fit, pooling cells with expected count < 5."""
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


@pytest.fixture(scope="module")
def grmat():
    return synth.rmat_graph(10, seed=3, cache=False)


# ---------------------------------------------------------------- exact refs
def test_dense_ppr_two_node_closed_form():
    gold = json.load(open(os.path.join(GOLDEN, "ppr_two_node.json")))
    g = _graph(gold["graph"])
    Pi = exact.dense_ppr(g, gold["alpha"])
    np.testing.assert_allclose(Pi[0], gold["pi_row0"], rtol=0, atol=1e-15)


def test_power_iteration_agrees_with_dense(g1k, pi1k):
    pe = exact.power_iteration(g1k, 0, ALPHA, iters=100)
    assert np.abs(pe - pi1k[0]).sum() <= (1 - ALPHA) ** 100 + 1e-12


# ---------------------------------------------------------------- Philox
def test_philox_word_statistics():
    N = 1 << 16
    ctr = np.zeros((N, 4), np.uint32)
    ctr[:, 0] = np.arange(N)
    ctr[:, 1] = 7
    ctr[:, 2] = 3
    y = oracle.philox(ctr, [5, 9])
    for w in range(4):
        hist = np.bincount(y[:, w] >> 24, minlength=256)
        assert st.chisquare(hist).pvalue > 1e-6
        bits = ((y[:, w][:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
        assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(N))
    # joint distribution of two words' top nibbles is uniform (no coupling)
    joint = np.bincount((y[:, 0] >> 28) * 16 + (y[:, 1] >> 28), minlength=256)
    assert st.chisquare(joint).pvalue > 1e-6
    assert len(np.unique(y.view(np.dtype((np.void, 16))))) == N


def test_philox_avalanche():
    rng = np.random.default_rng(4)
    base = rng.integers(0, 2**32, size=(256, 4), dtype=np.uint64).astype(np.uint32)
    y0 = oracle.philox(base, [11, 13])
    flips = []
    for bit in range(128):
        c = base.copy()
        c[:, bit // 32] ^= np.uint32(1 << (bit % 32))
        d = oracle.philox(c, [11, 13]) ^ y0
        flips.append(np.unpackbits(d.view(np.uint8), axis=1).sum(1).mean())
    flips = np.array(flips)
    assert abs(flips.mean() - 64) < 1.0
    assert flips.min() > 56


# ---------------------------------------------------------------- constants
@pytest.mark.parametrize("n,m,eps", [(1000, 10000, 0.5), (1 << 20, 16588107, 0.5),
                                     (1 << 26, 1 << 30, 0.1)])
def test_rmax_is_lagrange_optimum(n, m, eps):
    # eqn:rmax minimises 1/r + m r omega_unit (section 3.2), i.e. r = 1/sqrt(m omega_unit)
    c = oracle.constants(m, ALPHA, eps, 1.0 / n, 1.0 / n)
    assert m * c["rmax"] <= 1.0
    assert c["rmax"] == pytest.approx(1.0 / math.sqrt(m * c["omega_unit"]), rel=1e-14)


def test_rmax_case_two():
    # section 3.2, case 2: m r_max > 1 -> r_max = eps^2 delta / (c L) = 1 / omega_unit
    c = oracle.constants(10**9, ALPHA, 0.5, 1e-3, 1e-3)
    assert c["rmax"] == pytest.approx(1.0 / c["omega_unit"], rel=1e-14)
    assert 10**9 / math.sqrt(10**9 * c["omega_unit"]) > 1.0


@pytest.mark.parametrize("eps,delta,pf", [(0.5, 1e-3, 1e-3), (0.1, 1e-6, 1e-4),
                                          (0.3, 2.0**-20, 2.0**-20)])
def test_omega_meets_lemma2_bound(eps, delta, pf):
    # Lemma 1 / Lemma 2: with omega = r_sum omega_unit the failure bound at
    # pi = delta is exactly p_f (natural log).
    c = oracle.constants(12345, ALPHA, eps, delta, pf)
    for r_sum in (1.0, 0.3, 1e-3):
        omega = r_sum * c["omega_unit"]
        bound = 2 * math.exp(-(eps**2) * omega * delta / (r_sum * (2 + 2 * eps / 3)))
        assert bound == pytest.approx(pf, rel=1e-12)


def test_t_alpha_floor():
    for a in (0.2, 0.15, 0.5, 1e-3):
        t = oracle.constants(100, a, 0.5, 0.01, 0.01)["t_alpha"]
        assert t <= a * 2**32 < t + 1


# ---------------------------------------------------------------- push
def test_push_golden_synchronous_rounds():
    gold = json.load(open(os.path.join(GOLDEN, "push_sync_tiny.json")))
    g = _graph(gold["graph"])
    res = oracle.push(g, gold["source"], gold["alpha"], gold["rmax"], log_frontiers=True)
    assert res["rounds"] == gold["rounds"]
    assert list(res["round_sizes"]) == gold["round_sizes"]
    assert [list(f) for f in res["frontiers"]] == gold["frontiers"]
    np.testing.assert_allclose(res["q"], gold["reserve"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(res["r"], gold["residue"], rtol=0, atol=1e-15)


def _check_push(g, Pi, s, rmax):
    res = oracle.push(g, s, ALPHA, rmax)
    r, q = res["r"], res["q"]
    deg = g.degrees()
    # eqn:layerppr: pi(s,t) = q(t) + sum_v r(v) pi(v,t)
    np.testing.assert_allclose(q + r @ Pi, Pi[s], rtol=0, atol=1e-12)
    # each push moves alpha x to q and (1-alpha) x to neighbours: mass is kept
    assert q.sum() + r.sum() == pytest.approx(1.0, abs=1e-12)
    # termination test of Algorithm 1
    assert np.all(r <= rmax * deg)
    assert np.all(r >= 0) and np.all(q >= 0)
    assert np.all(q <= Pi[s] + 1e-15)
    # Forward Push runs in O(1/r_max): each push of v has d(v) < x_v / r_max and
    # the pushed mass sum x_v equals sum q / alpha.
    assert res["edge_ops"] < q.sum() / (ALPHA * rmax) + 1
    return res


@pytest.mark.parametrize("s", [0, 17, 999])
@pytest.mark.parametrize("rmax", [3.754e-5, 1e-3, 1e-6])
def test_push_invariant_uniform(g1k, pi1k, s, rmax):
    _check_push(g1k, pi1k, s, rmax)


def test_push_invariant_rmat(grmat):
    Pi = exact.dense_ppr(grmat, ALPHA)
    deg = grmat.degrees()
    for s in (int(np.argmax(deg)), 5, 700):
        for rmax in (1e-4, 1e-6):
            _check_push(grmat, Pi, s, rmax)


def test_push_rmax_to_zero_is_exact(g1k, pi1k):
    # section 2.2: Forward Push computes exact PPR as r_max -> 0; the remaining
    # L1 error is exactly r_sum, which is at most m r_max
    rmax = 1e-13
    res = oracle.push(g1k, 0, ALPHA, rmax)
    err = np.abs(pi1k[0] - res["q"]).sum()
    assert err == pytest.approx(res["r"].sum(), abs=1e-12)
    assert res["r"].sum() <= g1k.m * rmax


# ---------------------------------------------------------------- plan
def test_plan_counts_and_bounds(g1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    res = oracle.push(g1k, 0, ALPHA, c["rmax"])
    pv, po, pw = oracle.plan(res["r"], c["omega_unit"])
    r = res["r"]
    assert np.array_equal(pv, np.flatnonzero(r > 0))
    x = r[pv] * c["omega_unit"]
    om = po.astype(np.float64)
    assert np.all(om - 1 < x) and np.all(x <= om)
    # eqn:index-rwnum: omega_v <= ceil(d(v) r_max omega_unit)
    deg = g1k.degrees()[pv]
    assert np.all(om <= np.ceil(deg * c["rmax"] * c["omega_unit"]))
    # sum of walk weights equals r_sum (Algorithm 2's increments)
    assert (om * pw).sum() == pytest.approx(r.sum(), rel=1e-12)
    # section 3.2: r_sum <= m r_max, so W <= m r_max omega_unit + |supp r|
    assert om.sum() <= g1k.m * c["rmax"] * c["omega_unit"] + len(pv)


# ---------------------------------------------------------------- walks
def _one_entry_walks(g, v, omega, seed=0, source=0, endpoints=True):
    t_alpha = oracle.constants(g.m, ALPHA, 0.5, 0.01, 0.01)["t_alpha"]
    return oracle.walks(g, source, seed, t_alpha, np.array([v], np.int32),
                        np.array([omega], np.uint64), np.array([1.0 / omega]),
                        endpoints=endpoints)


def test_walk_length_is_geometric():
    # directed cycle of length L: the end point encodes the walk length mod L
    L = 64
    g = Graph(np.arange(L + 1, dtype=np.int32), ((np.arange(L) + 1) % L).astype(np.int32))
    W = 200000
    res = _one_entry_walks(g, 0, W)
    hist = np.bincount(res["endpoints"], minlength=L)
    ell = np.arange(L)
    p = ALPHA * (1 - ALPHA) ** ell / (1 - (1 - ALPHA) ** L)
    assert _chi2_pvalue(hist, p * W) > 1e-6
    mean_len = res["steps"] / W
    assert abs(mean_len - (1 - ALPHA) / ALPHA) < 5 * math.sqrt((1 - ALPHA) / ALPHA**2 / W)


def test_walk_neighbour_choice_is_uniform():
    # star: 0 -> 1..d, every leaf -> 0. A walk from 0 that ends after exactly
    # one move ends at a uniformly random leaf; all leaves are symmetric.
    d = 37
    rowptr = np.concatenate([[0], d + np.arange(0, d + 1)]).astype(np.int32)
    colidx = np.concatenate([np.arange(1, d + 1), np.zeros(d)]).astype(np.int32)
    g = Graph(rowptr, colidx)
    assert oracle.validate(g) == 0
    res = _one_entry_walks(g, 0, 300000)
    hist = np.bincount(res["endpoints"], minlength=d + 1)
    assert st.chisquare(hist[1:]).pvalue > 1e-6
    # P(end at 0) = alpha / (1 - (1-alpha)^2) on this bipartite star
    p0 = ALPHA / (1 - (1 - ALPHA) ** 2)
    assert abs(hist[0] / 300000 - p0) < 5 * math.sqrt(p0 * (1 - p0) / 300000)


def test_walk_endpoints_follow_ppr_row(g1k, pi1k):
    v, W = 3, 400000
    res = _one_entry_walks(g1k, v, W)
    hist = np.bincount(res["endpoints"], minlength=g1k.n)
    assert _chi2_pvalue(hist, pi1k[v] * W) > 1e-6


def test_walks_are_keyed_by_start_and_index(g1k):
    a = _one_entry_walks(g1k, 5, 10)
    b = _one_entry_walks(g1k, 5, 4)
    assert np.array_equal(a["endpoints"][:4], b["endpoints"])
    c = _one_entry_walks(g1k, 5, 10, seed=1)
    assert not np.array_equal(a["endpoints"], c["endpoints"])


def test_walk_weight_lands_at_the_end_point(g1k):
    # Algorithm 2: a walk from v that ends at t adds v's weight to pi_hat(t);
    # with one plan entry, the weight at each node is its end-point count
    # times the entry's weight, and the recorded end points give the counts
    v, W, w = 11, 5000, 0.375
    t_alpha = oracle.constants(g1k.m, ALPHA, 0.5, 0.01, 0.01)["t_alpha"]
    res = oracle.walks(g1k, 0, 0, t_alpha, np.array([v], np.int32),
                       np.array([W], np.uint64), np.array([w]), endpoints=True)
    cnt = np.bincount(res["endpoints"], minlength=g1k.n)
    assert np.array_equal(res["cnt"], cnt)
    assert np.count_nonzero(cnt) > 100
    np.testing.assert_allclose(res["acc"], cnt * w, rtol=1e-12, atol=0)


def test_walk_totals(g1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    res = oracle.push(g1k, 0, ALPHA, c["rmax"])
    pv, po, pw = oracle.plan(res["r"], c["omega_unit"])
    wk = oracle.walks(g1k, 0, 7, c["t_alpha"], pv, po, pw)
    assert int(wk["cnt"].sum()) == int(po.sum()) == wk["walks"]
    assert wk["acc"].sum() == pytest.approx(res["r"].sum(), rel=1e-12)


# ---------------------------------------------------------------- estimator
def test_pi_hat_sums_to_one(g1k):
    out = oracle.fora(g1k, 0, k=50, seed=3)
    assert out["pi"].sum() == pytest.approx(1.0, abs=1e-12)


def test_monte_carlo_special_case(g1k):
    # r_max >= 1 / d(s): no push happens and Algorithm 2 is plain MC with
    # ceil(omega_unit) walks from s (section 2.2).
    out = oracle.fora(g1k, 0, k=50, seed=0, rmax=1.0)
    assert out["rounds"] == 0
    pv, po, pw = out["plan"]
    assert list(pv) == [0]
    assert int(po[0]) == math.ceil(out["consts"]["omega_unit"])
    assert np.all(out["q"] == 0)


@pytest.fixture(scope="module")
def repeated(g1k):
    R = 300
    return np.stack([oracle.fora(g1k, 0, k=50, seed=s)["pi"] for s in range(R)])


def test_estimator_is_unbiased(repeated, pi1k):
    # eqn:ss-exp with eqn:layerppr: E[pi_hat] = pi
    R = repeated.shape[0]
    mean = repeated.mean(0)
    sd = repeated.std(0, ddof=1)
    mask = pi1k[0] >= 1e-3
    z = (mean[mask] - pi1k[0][mask]) / (sd[mask] / math.sqrt(R))
    assert np.max(np.abs(z)) < 5.5
    assert np.abs(mean - pi1k[0]).sum() < 0.01


def test_eps_guarantee_and_lemma1_tail(repeated, pi1k):
    R = repeated.shape[0]
    eps, delta, pf = 0.5, 1e-3, 1e-3
    pi = pi1k[0]
    mask = pi >= delta
    fails = (np.abs(repeated[:, mask] - pi[mask]) > eps * pi[mask]).sum()
    trials = R * mask.sum()
    assert fails <= st.binom(trials, pf).ppf(1 - 1e-6)
    # eqn:relative-error at a tighter level e = 0.1 for nodes with pi >= 0.01
    c = oracle.constants(10000, ALPHA, eps, delta, pf)
    e = 0.1
    big = np.flatnonzero(pi >= 0.01)
    out = oracle.fora(synth.uniform_out_graph(1000, 10, seed=1), 0, k=50, seed=0)
    r_sum = out["r_sum"]
    omega = r_sum * c["omega_unit"]
    for t in big:
        bound = 2 * math.exp(-(e**2) * omega * pi[t] / (r_sum * (2 + 2 * e / 3)))
        freq = (np.abs(repeated[:, t] - pi[t]) >= e * pi[t]).mean()
        assert freq <= min(1.0, bound) + 4 * math.sqrt(0.25 / R)


# ---------------------------------------------------------------- top-k
def test_topk_matches_sort():
    rng = np.random.default_rng(8)
    pi = rng.integers(0, 50, size=5000).astype(np.float64) / 64.0  # many ties, zeros
    for k in (1, 50, 500, 5000):
        ids, vals = oracle.topk(pi, k)
        order = np.lexsort((np.arange(pi.size), -pi))[:k]
        assert np.array_equal(ids, order)
        assert np.array_equal(vals, pi[order])


# ---------------------------------------------------------------- validation
def test_validate_rejects_malformed():
    ok = Graph(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32))
    assert oracle.validate(ok) == 0
    assert oracle.validate(Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32))) == -3
    assert oracle.validate(Graph(np.array([0, 1, 2], np.int32), np.array([1, 2], np.int32))) == -2
    assert oracle.validate(Graph(np.array([0, 2, 1], np.int32), np.array([1], np.int32))) == -1


# ---------------------------------------------------------------- generators
def test_uniform_graph_shape():
    g = synth.uniform_out_graph(1000, 10, seed=1)
    assert g.m == 10000
    for v in range(g.n):
        row = g.colidx[g.rowptr[v]:g.rowptr[v + 1]]
        assert len(set(row.tolist())) == 10 and v not in row
        assert np.all(np.diff(row) > 0)
    h = synth.uniform_out_graph(1000, 10, seed=1)
    assert np.array_equal(g.colidx, h.colidx)


def test_rmat_graph_shape(grmat):
    g = grmat
    deg = g.degrees()
    assert deg.min() >= 1
    src = np.repeat(np.arange(g.n), deg)
    assert np.all(src != g.colidx)
    key = src.astype(np.int64) * g.n + g.colidx
    assert np.all(np.diff(key) > 0)  # sorted, no duplicates
    extra = deg - g.deg_before_fixup
    assert set(np.unique(extra).tolist()) <= {0, 1}
    assert np.all((extra == 1) == (g.deg_before_fixup == 0))
    h = synth.rmat_graph(10, seed=3, cache=False)
    assert np.array_equal(g.colidx, h.colidx)
    s = synth.sources_uniform(g, 50, seed=1)
    assert np.all(g.deg_before_fixup[s] >= 1) and len(np.unique(s)) == 50
