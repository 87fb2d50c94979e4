"""Pins of the oracle's top-k FORA (Algorithm 5, section 5.2). CPU only.

Definition 2 is checked against the exact PPR of a dense solve over many
seeds (the frequency of violations must stay within the failure budget),
and the stopping threshold against Lemma 3's range for the true k-th PPR."""
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


def test_delta_sequence():
    assert oracle.topk_deltas(1000, 10) == [0.1 / 2**i for i in range(7)] + [1e-3]
    assert oracle.topk_deltas(1000, 1000) == [1e-3]
    d = oracle.topk_deltas(2**20, 500)
    assert d[0] == 1 / 500 and d[-1] == 2.0**-20 and all(b == a / 2 for a, b in zip(d[:-2], d[1:-1]))


def test_iterations_hold_the_union_bound(g1k):
    # Algorithm 5's guarantee (section 5.2) is a union bound: each iteration
    # keeps every node with pi >= delta within eps/2 of its PPR except with
    # probability p_f / (n log2(n/k)), so that over the n nodes and the
    # log2(n/k) halvings of delta the failure probability is p_f. Lemma 2's
    # bound at relative error eps/2, the iteration's delta and its omega_unit
    # is that per-node probability.
    n, k, eps, pf = g1k.n, 50, 0.5, 1.0 / g1k.n
    out = oracle.fora_topk(g1k, 0, k, eps=eps, pf=pf, seed=1)
    assert len(out["trace"]) >= 2
    e2 = eps / 2
    for it in out["trace"]:
        fail = 2 * math.exp(-(e2**2) * it["delta"] * it["omega_unit"] / (2 + 2 * e2 / 3))
        assert fail * n * math.log2(n / k) == pytest.approx(pf, rel=1e-9)


@pytest.mark.parametrize("k", [5, 50])
def test_definition_2_and_stopping_threshold(g1k, pi1k, k):
    s, eps = 0, 0.5
    pi = pi1k[s]
    order = np.sort(pi)[::-1]
    R = 40
    viol = trials = 0
    deltas = []
    for seed in range(R):
        out = oracle.fora_topk(g1k, s, k, eps=eps, seed=100 * seed)
        ids = out["topk_ids"]
        est = out["pi"][ids]
        for i in range(k):
            if order[i] > 1.0 / g1k.n:
                trials += 1
                ok = est[i] >= (1 - eps) * pi[ids[i]] and pi[ids[i]] >= (1 - eps) * order[i]
                viol += not ok
        deltas.append(out["delta"])
        last = out["trace"][-1]
        assert last["kth"] >= last["bound"] or out["delta"] == 1.0 / g1k.n
        assert all(t["kth"] < t["bound"] for t in out["trace"][:-1])
    assert viol <= st.binom(trials, 1.0 / g1k.n).ppf(1 - 1e-6)
    # Lemma 3: the run stops with delta <= pi(v_k*) but not far below it
    deltas = np.array(deltas)
    assert np.mean(deltas <= order[k - 1]) >= 0.9
    assert np.all(deltas >= order[k - 1] / 16)
