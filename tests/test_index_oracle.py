"""Pins of FORA+ (section 3.3) in the oracle: walks taken from an index
shared by all sources. CPU only.

The estimator stays unbiased over index draws and keeps the eps guarantee;
the index holds omega_max(v) = ceil(d(v) r_max omega_unit) end points per
node, within Lemma 4's bound, and its end points follow each node's PPR row."""
import math

import numpy as np
import pytest
import scipy.stats as st

import oracle
import synth
from oracle import exact

ALPHA = 0.2


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def pi1k(g1k):
    return exact.dense_ppr(g1k, ALPHA)


def test_index_size_and_contents(g1k, pi1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    wpd = c["rmax"] * c["omega_unit"]
    idx = oracle.build_index(g1k, ALPHA, wpd, (7, 9))
    total = int(idx["off"][-1])
    # eqn:index-rwnum, and Lemma 4's n + m r_max omega_unit bound
    assert np.array_equal(idx["omega_max"], np.ceil(g1k.degrees() * wpd).astype(np.uint64))
    assert total <= g1k.n + g1k.m * wpd
    # every push leaves r(v) <= r_max d(v), so the index covers every plan
    res = oracle.push(g1k, 0, ALPHA, c["rmax"])
    pv, po, _ = oracle.plan(res["r"], c["omega_unit"])
    assert np.all(po <= idx["omega_max"][pv])
    # pooled end points of node 3's index walks follow its PPR row
    v = 3
    big = oracle.build_index(g1k, ALPHA, 400.0, (7, 9))
    ends = big["dest"][int(big["off"][v]):int(big["off"][v + 1])]
    hist = np.bincount(ends, minlength=g1k.n)
    exp_ = pi1k[v] * len(ends)
    keep = exp_ >= 5
    o = np.append(hist[keep], hist[~keep].sum())
    e = np.append(exp_[keep], exp_[~keep].sum())
    assert st.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-6


def test_index_walks_are_the_query_walks(g1k):
    # FORA+ reads the first omega_v stored end points of v: the same walks a
    # query keyed by the index key would run
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    idx = oracle.build_index(g1k, ALPHA, c["rmax"] * c["omega_unit"], (7, 9))
    out = oracle.fora(g1k, 0, k=50, delta=1e-3, pf=1e-3, walk_key=(7, 9))
    pv, po, pw = out["plan"]
    cnt = np.zeros(g1k.n, np.uint64)
    for v, o in zip(pv, po):
        ends = idx["dest"][int(idx["off"][v]):int(idx["off"][v]) + int(o)]
        np.add.at(cnt, ends, 1)
    assert np.array_equal(cnt, out["cnt"])


@pytest.fixture(scope="module")
def over_index_keys(g1k):
    R = 300
    return np.stack([oracle.fora(g1k, 0, k=50, seed=0, delta=1e-3, pf=1e-3,
                                 walk_key=(1000 + r, 5))["pi"] for r in range(R)])


def test_unbiased_over_index_draws(over_index_keys, pi1k):
    R = over_index_keys.shape[0]
    mean = over_index_keys.mean(0)
    sd = over_index_keys.std(0, ddof=1)
    mask = (pi1k[0] >= 1e-3) & (sd > 0)
    z = (mean[mask] - pi1k[0][mask]) / (sd[mask] / math.sqrt(R))
    assert np.max(np.abs(z)) < 5.5


def test_guarantee_over_index_draws(over_index_keys, pi1k):
    R = over_index_keys.shape[0]
    pi = pi1k[0]
    mask = pi >= 1e-3
    fails = (np.abs(over_index_keys[:, mask] - pi[mask]) > 0.5 * pi[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1e-3).ppf(1 - 1e-6)
