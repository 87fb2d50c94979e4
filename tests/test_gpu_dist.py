"""FORA for source distributions and global PageRank on the GPU against the
oracle: the device's push of the distribution against the oracle replaying
its frontiers (r and q to 1e-5 element by element), walk end-point counts and
moves exactly equal to the oracle's walks on the device's residues, the
estimate, the selection, and the eps guarantee for global PageRank; invalid
distributions are rejected."""
import numpy as np
import pytest
import scipy.stats as st

import exactcmp
import oracle
import synth
from oracle import exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora  # noqa: E402

ALPHA = 0.2
WC = fora.FORA_WALK_COUNTS


def close(g, o, rtol=1e-5, atol=1e-12):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return np.abs(g - o) <= rtol * np.abs(o) + atol


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def G1k(g1k):
    G = fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)
    yield G
    G.close()


@pytest.fixture(scope="module")
def grmat():
    return synth.rmat_graph(12, seed=12, cache=False)


@pytest.fixture(scope="module")
def Grmat(grmat):
    G = fora.Graph.from_numpy(grmat.rowptr, grmat.colidx)
    yield G
    G.close()


def _sigma(n, seed, support):
    # a random distribution on `support` nodes whose values are exact in
    # FP32, hence in the residues' fixed point: both sides start from them
    rng = np.random.default_rng(seed)
    v = rng.choice(n, support, replace=False)
    w = rng.integers(1, 1 << 10, support).astype(np.float64)
    s = np.zeros(n)
    s[v] = w / w.sum()
    return s.astype(np.float32).astype(np.float64)


def _run(G, g, sigmas, seeds, k=50, **kw):
    B = len(sigmas)
    qs = fora.make_queries([0] * B, k=k, seed=seeds, n=g.n, flags=WC, **kw)
    ws = fora.workspace(G, B)
    sig = torch.as_tensor(np.stack(sigmas), dtype=torch.float64, device="cuda")
    res = fora.fora_dist_batch(G, qs, sig, ws=ws, stats=True)
    rows = {k_: t.cpu().numpy().copy() for k_, t in fora.fora_workspace_views(G, B, ws).items()}
    return res, rows


def _compare(g, G, res, rows, i, sig, seed, ref=None):
    """Row i against the oracle: the device's push of sigma (rerun alone
    with its frontiers logged, equal to the row bit for bit) against the
    oracle replaying those frontiers from sigma; walks on the device's
    residues exactly as the oracle's (keyed by the distribution key); the
    estimate and the selection from them. Where the oracle's own free run
    keeps every residue clear of its threshold, it agrees as well."""
    st_ = res.stats[i]
    p = fora.fora_push_only(G, 0, ALPHA, st_["rmax"], log_frontiers=True,
                            sigma=torch.as_tensor(sig, device="cuda"))
    assert np.array_equal(p["r_fx"].cpu().numpy(), rows["residue_fx"][i])
    assert np.array_equal(p["q"].cpu().numpy(), rows["reserve"][i])
    assert p["stats"]["rounds"] == st_["rounds"] and p["stats"]["edge_ops"] == st_["edge_ops"]
    exactcmp.check_push(g, 0, ALPHA, st_["rmax"], p["frontiers"], rows["residue"][i],
                        rows["reserve"][i], r0=sig)
    w = exactcmp.oracle_walks_on(g, rows["residue"][i], st_["omega_unit"], oracle.DIST_KEY0,
                                 seed, st_["t_alpha"])
    assert w["walks"] == st_["walks"]
    exactcmp.check_walks(w, rows["walk_count"][i], st_["steps"], rows["walk_weight_fx"][i])
    acc = rows["walk_weight_fx"][i].view(np.uint64).astype(np.float64) * 2.0**-62
    want = (rows["reserve"][i].astype(np.float64) + acc).astype(np.float32)
    assert np.array_equal(rows["pi_hat"][i], want)
    order = np.lexsort((np.arange(g.n), -rows["pi_hat"][i]))[:res.ids.shape[1]]
    assert np.array_equal(res.ids[i].cpu().numpy(), order)
    if ref is not None and ref["min_margin"] > 1e-5:
        assert st_["rounds"] == ref["rounds"] and st_["edge_ops"] == ref["edge_ops"]
        assert np.all(close(rows["reserve"][i], ref["q"]))
        assert st_["steps"] == ref["steps"] and st_["walks"] == ref["walks"]


def test_distributions_match_oracle(g1k, G1k):
    n = g1k.n
    sigmas = [_sigma(n, 1, 50), _sigma(n, 2, 3), np.where(np.arange(n) < 512, 1.0 / 512, 0.0)]
    seeds = [4, 5, 6]
    res, rows = _run(G1k, g1k, sigmas, seeds, delta=1e-3, pf=1e-3)
    for i, (sg, sd) in enumerate(zip(sigmas, seeds)):
        ref = oracle.fora_dist(g1k, sg, alpha=ALPHA, k=50, seed=sd, delta=1e-3, pf=1e-3)
        _compare(g1k, G1k, res, rows, i, sg, sd, ref)


def test_uniform_distribution_on_rmat(grmat, Grmat):
    # global PageRank's start: every node holds 1/n (a power of two here, so
    # exact in the residues' fixed point); round 0's frontier is every node with d(v) < 1/(n r_max)
    n = grmat.n
    sig = np.full(n, 1.0 / n)
    c = oracle.constants(grmat.m, ALPHA, 0.5, 1.0 / n, 1.0 / n)
    for rmax in (c["rmax"], c["rmax"] / 8):
        ref = oracle.fora_dist(grmat, sig, alpha=ALPHA, k=100, seed=9, rmax=rmax,
                               log_frontiers=True)
        res, rows = _run(Grmat, grmat, [sig], [9], k=100, rmax=rmax)
        first = np.flatnonzero(sig > rmax * grmat.degrees())
        assert np.array_equal(np.sort(ref["frontiers"][0]), first)
        _compare(grmat, Grmat, res, rows, 0, sig, 9, ref)


def test_point_mass_pushes_like_the_single_source_query(g1k, G1k):
    sig = np.zeros(g1k.n)
    sig[17] = 1.0
    res, rows = _run(G1k, g1k, [sig], [3], delta=1e-3, pf=1e-3)
    one = fora.fora_ssppr(G1k, 17, k=50, seed=3, delta=1e-3, pf=1e-3, stats=True)
    assert res.stats[0]["rounds"] == one.stats["rounds"]
    assert res.stats[0]["edge_ops"] == one.stats["edge_ops"]
    ref = oracle.fora(g1k, 17, k=50, seed=3, delta=1e-3, pf=1e-3,
                      walk_key=(oracle.DIST_KEY0, 3))
    _compare(g1k, G1k, res, rows, 0, sig, 3, ref)


def test_pagerank_keeps_the_guarantee(g1k, G1k):
    n = g1k.n
    pr = exact.dense_ppr(g1k, ALPHA).mean(0)
    R, eps = 16, 0.5
    est = []
    ws = fora.workspace(G1k, 1)
    for s in range(R):
        fora.pagerank(G1k, alpha=ALPHA, eps=eps, k=10, seed=s, ws=ws)
        est.append(fora.fora_workspace_views(G1k, 1, ws)["pi_hat"][0].cpu().numpy().astype(
            np.float64))
    est = np.stack(est)
    mask = pr >= 1.0 / n
    fails = (np.abs(est[:, mask] - pr[mask]) > eps * pr[mask]).sum()
    assert fails <= st.binom(R * mask.sum(), 1.0 / n).ppf(1 - 1e-6)
    assert np.abs(est.mean(0) - pr).sum() < 0.05


def test_invalid_distributions_are_rejected(g1k, G1k):
    n = g1k.n
    qs = fora.make_queries([0], k=10, n=n)
    for bad in (-1e-3, float("nan"), float("inf"), 1.5):
        sig = np.full((1, n), 1.0 / n)
        sig[0, 7] = bad
        with pytest.raises(fora.FORAError) as ei:
            fora.fora_dist_batch(G1k, qs, torch.as_tensor(sig, device="cuda"))
        assert ei.value.code == fora.FORA_E_ARG
    with pytest.raises(ValueError):
        fora.fora_dist_batch(G1k, qs, torch.zeros((2, n), dtype=torch.float64, device="cuda"))
    # the next good call works
    r = fora.fora_dist_batch(G1k, qs, torch.full((1, n), 1.0 / n, dtype=torch.float64,
                                                 device="cuda"), stats=True)
    assert r.stats[0]["walks"] > 0
