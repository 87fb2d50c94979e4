"""Pins of the oracle's source-distribution FORA (sections 6.2 and 6.3, the
extension to source distributions and global PageRank). CPU only.

The extension only changes Algorithm 1's start (r = sigma instead of e_s),
so it is pinned by: the point mass sigma = e_s reducing bit for bit to the
single-source oracle with the same walk key; the invariant
pi(sigma, t) = q(t) + sum_v r(v) pi(v, t) and mass conservation against the
dense solve (pi(sigma, .) = sigma Pi); unbiasedness over seeds; and, for
global PageRank (sigma uniform), the eps guarantee against the PageRank
vector of the dense solve."""
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


def _sigma(n, seed, support=50):
    # a random distribution on `support` nodes, values exact in FP32
    rng = np.random.default_rng(seed)
    v = rng.choice(n, support, replace=False)
    w = rng.integers(1, 1 << 10, support).astype(np.float64)
    s = np.zeros(n)
    s[v] = w / w.sum()
    return s.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("src,seed", [(0, 1), (5, 2), (999, 3)])
def test_point_mass_is_the_single_source_query(g1k, src, seed):
    sig = np.zeros(g1k.n)
    sig[src] = 1.0
    a = oracle.fora_dist(g1k, sig, alpha=ALPHA, k=50, seed=seed, delta=1e-3, pf=1e-3)
    b = oracle.fora(g1k, src, alpha=ALPHA, k=50, seed=seed, delta=1e-3, pf=1e-3,
                    walk_key=(oracle.DIST_KEY0, seed))
    assert a["rounds"] == b["rounds"] and a["edge_ops"] == b["edge_ops"]
    np.testing.assert_array_equal(a["r"], b["r"])
    np.testing.assert_array_equal(a["q"], b["q"])
    np.testing.assert_array_equal(a["cnt"], b["cnt"])
    np.testing.assert_array_equal(a["pi"], b["pi"])
    np.testing.assert_array_equal(a["topk_ids"], b["topk_ids"])


@pytest.mark.parametrize("seed", [0, 1])
def test_push_from_a_distribution_keeps_the_invariant(g1k, pi1k, seed):
    sig = _sigma(g1k.n, seed)
    for rmax in (1e-3, 1e-4, 1e-6):
        out = oracle.fora_dist(g1k, sig, alpha=ALPHA, k=50, seed=seed, rmax=rmax)
        r, q = out["r"], out["q"]
        # pi(sigma, .) = sigma Pi = q + r Pi, and no mass is lost
        np.testing.assert_allclose(q + r @ pi1k, sig @ pi1k, atol=1e-12)
        assert q.sum() + r.sum() == pytest.approx(sig.sum(), abs=1e-12)
        # termination: every residue is at or below its threshold
        assert np.all(r <= rmax * g1k.degrees() * (1 + 1e-12))
        assert out["rounds"] > 0 and out["r_sum"] == pytest.approx(r.sum())


def test_uniform_sigma_starts_with_every_node_over_threshold(g1k):
    # r = 1/n everywhere and every d(v) = 10: r_max below 1/(10 n) puts all n
    # nodes in the first frontier, r_max above it none (pure Monte Carlo)
    n = g1k.n
    sig = np.full(n, 1.0 / n)
    low = oracle.fora_dist(g1k, sig, rmax=0.9 / (10 * n), k=10, log_frontiers=True)
    assert low["round_sizes"][0] == n
    np.testing.assert_array_equal(low["frontiers"][0], np.arange(n))
    high = oracle.fora_dist(g1k, sig, rmax=1.1 / (10 * n), k=10)
    assert high["rounds"] == 0 and np.array_equal(high["r"], sig)
    # each node then starts ceil(omega_unit / n) walks
    pv, po, _ = high["plan"]
    assert len(pv) == n and np.all(po == math.ceil(high["consts"]["omega_unit"] / n))


def test_distribution_estimate_is_unbiased(g1k, pi1k):
    sig = _sigma(g1k.n, 7)
    truth = sig @ pi1k
    R = 200
    est = np.stack([oracle.fora_dist(g1k, sig, alpha=ALPHA, k=10, seed=s, delta=1e-3,
                                     pf=1e-3)["pi"] for s in range(R)])
    mean, sd = est.mean(0), est.std(0, ddof=1)
    mask = (truth >= 1e-3) & (sd > 0)
    z = (mean[mask] - truth[mask]) / (sd[mask] / math.sqrt(R))
    assert np.max(np.abs(z)) < 5.5
    assert np.abs(mean - truth).sum() < 0.01


def test_global_pagerank_keeps_the_guarantee(g1k, pi1k):
    n = g1k.n
    pr = pi1k.mean(0)  # PageRank = (1/n) 1^T Pi
    assert pr.sum() == pytest.approx(1.0, abs=1e-12)
    R, eps, delta = 40, 0.5, 1.0 / n
    est = np.stack([oracle.fora_dist(g1k, np.full(n, 1.0 / n), alpha=ALPHA, eps=eps, k=10,
                                     seed=s)["pi"] for s in range(R)])
    mask = pr >= delta
    fails = (np.abs(est[:, mask] - pr[mask]) > eps * pr[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1.0 / n).ppf(1 - 1e-6)
