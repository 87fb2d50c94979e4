"""Pins of the learned-r_max reference (CPU only).

The FP64 MLP reference is checked against finite differences, closed forms
of GELU and of Adam's first step, hand-computed BF16 roundings, features
worked by hand on a small graph, and Lemma 2's claim that the eps guarantee
holds whatever r_max is.
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import oracle
import synth
from oracle import exact, mlp
from synth.graphs import Graph


def _params(seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, mlp.NPARAMS)
    p[mlp.MU:mlp.MU + 7] = rng.normal(0, 1, 7)
    p[mlp.SIG:mlp.SIG + 7] = rng.uniform(0.5, 2.0, 7)
    return p


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(1)
    X = rng.normal(0, 1, (37, 7))
    t = rng.normal(0, 1, 37)
    g = mlp.backward(p, X, t)
    assert np.all(g[:mlp.TRAIN0] == 0)
    idx = np.concatenate([rng.choice(np.arange(mlp.TRAIN0, mlp.NPARAMS), 200, replace=False),
                          [mlp.B3, mlp.B1, mlp.W3]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, X, t) - mlp.loss(pm, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gelu_closed_forms():
    z = np.linspace(-6, 6, 101)
    # z Phi(z) - (-z) Phi(-z) = z because Phi(z) + Phi(-z) = 1
    np.testing.assert_allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    assert mlp.gelu(0.0) == 0.0 and mlp.gelu_grad(0.0) == pytest.approx(0.5)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h),
                               atol=1e-8)


def test_adam_first_step_moves_by_lr():
    # bias correction makes the first step exactly lr * sign(g) (up to eps)
    p = _params(2)
    g = np.random.default_rng(3).normal(0, 1, mlp.NPARAMS)
    z = np.zeros(mlp.NPARAMS)
    p1, m1, v1 = mlp.adam(p, g, z, z, lr=0.01, b1=0.9, b2=0.999, eps=1e-12, step=1)
    sl = slice(mlp.TRAIN0, None)
    np.testing.assert_allclose(p1[sl] - p[sl], -0.01 * np.sign(g[sl]), rtol=1e-6)
    assert np.all(p1[:mlp.TRAIN0] == p[:mlp.TRAIN0])
    np.testing.assert_allclose(m1[sl], 0.1 * g[sl])
    np.testing.assert_allclose(v1[sl], 0.001 * g[sl] ** 2)


def test_bf16_rounding_cases():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -2.5, 3.0e38,
                  np.inf], np.float32)
    want = np.array([1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -2.5, 2.9975e38, np.inf], np.float32)
    got = mlp.bf16_round(x)
    np.testing.assert_array_equal(got[:5], want[:5])
    assert abs(got[5] - 3.0e38) / 3.0e38 < 2**-8
    assert np.isinf(got[6])


def test_features_hand_worked():
    # s = 0 -> {1, 2, 3}; d(1) = 1, d(2) = 2, d(3) = 4 (every node needs an edge)
    rowptr = np.array([0, 3, 4, 6, 10, 11, 12], np.int32)
    colidx = np.array([1, 2, 3, 0, 0, 1, 0, 1, 2, 4, 5, 0], np.int32)
    g = Graph(rowptr, colidx)
    assert oracle.validate(g) == 0
    alpha, rmax = 0.2, 0.1
    f = mlp.features(g, [0], alpha, 0.5, rmax)[0]
    share = 0.8 / 3
    # thresholds rmax*d(u) = 0.1, 0.2, 0.4: neighbours 1 and 2 are over
    assert f[0] == pytest.approx(math.log(3))
    assert f[1] == pytest.approx(math.log(1 + 2 + 4))
    assert f[2] == pytest.approx(2 * share)
    assert f[3] == pytest.approx(math.log(6)) and f[4] == pytest.approx(math.log(12))
    # a source that is not pushed at all (1 <= rmax * d(s)) has mass 0
    assert mlp.features(g, [0], alpha, 0.5, 0.5)[0][2] == 0.0


@pytest.mark.parametrize("mult", [0.25, 8.0])
def test_eps_guarantee_holds_for_other_rmax(mult):
    # Lemma 2 never uses r_max: the failure frequency stays within the bound
    g = synth.uniform_out_graph(1000, 10, seed=1)
    pi = exact.dense_ppr(g, 0.2)[0]
    c = oracle.constants(g.m, 0.2, 0.5, 1e-3, 1e-3)
    R = 60
    est = np.stack([oracle.fora(g, 0, k=50, seed=s, rmax=c["rmax"] * mult)["pi"]
                    for s in range(R)])
    mask = pi >= 1e-3
    fails = (np.abs(est[:, mask] - pi[mask]) > 0.5 * pi[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1e-3).ppf(1 - 1e-6)
    assert np.abs(est.mean(0) - pi).sum() < 0.02


def test_push_sweep_keeps_the_invariant_at_every_threshold():
    # Algorithm 1's loop from any state keeps eqn:layerppr and stops at the
    # termination test, so every point of the sweep is a valid push result
    g = synth.uniform_out_graph(1000, 10, seed=1)
    Pi = exact.dense_ppr(g, 0.2)
    deg = g.degrees()
    c = oracle.constants(g.m, 0.2, 0.5, 1e-3, 1e-3)
    mults = np.exp(np.linspace(math.log(8.0), math.log(0.25), 6))
    rms = c["rmax"] * mults
    for s in (0, 17):
        fresh = oracle.push(g, s, 0.2, rms[0])
        E_prev = 0
        for i in range(len(rms)):
            sw = oracle.push_sweep(g, s, 0.2, rms[:i + 1], c["omega_unit"])
            r, q = sw["r"], sw["q"]
            np.testing.assert_allclose(q + r @ Pi, Pi[s], atol=1e-12)
            assert q.sum() + r.sum() == pytest.approx(1.0, abs=1e-12)
            assert np.all(r <= rms[i] * deg)
            assert sw["E"][-1] >= E_prev
            E_prev = sw["E"][-1]
            assert sw["W"][-1] == np.ceil(r[r > 0] * c["omega_unit"]).sum()
            if i == 0:
                assert sw["E"][0] == fresh["edge_ops"]
                np.testing.assert_array_equal(r, fresh["r"])
