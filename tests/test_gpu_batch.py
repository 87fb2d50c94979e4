"""Batched queries, captured-graph replays and the autotuner (GPU).

Batched and graph-replayed results are compared with single-query eager calls
(bit for bit: residues are summed in fixed point and walks are keyed by
(source, seed, start, index, step), so no result depends on the batch, the
launch shape or the order of atomics) and with the oracle (the device's
frontiers replayed in FP64, walks on the device's residues exact).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import autotune, fora  # noqa: E402
import exactcmp  # noqa: E402

WC = fora.FORA_WALK_COUNTS  # the tests below compare per-node walk counts

RTOL, ATOL = 1e-5, 1e-12


def close(g, o, rtol=RTOL, atol=ATOL):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return np.abs(g - o) <= rtol * np.abs(o) + atol


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture
def G1k(g1k):
    G = fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)
    yield G
    G.close()


def _rows(G, B, ws):
    v = fora.fora_workspace_views(G, B, ws)
    return {k: t.cpu().numpy().copy() for k, t in v.items()}


def _same_query(a, b, i, j, omega_unit=None):
    """Row i of result a equals row j of result b, bit for bit."""
    for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
        assert np.array_equal(a[key][i], b[key][j]), key


def test_tuning_validation(G1k):
    t = G1k.get_tuning()
    assert t["walk_chunk"] % 64 == 0 and t["graph_rounds"] == 0
    for bad in (dict(walk_chunk=100), dict(walk_chunk=0), dict(walk_blocks_per_cu=0),
                dict(push_blocks_per_cu=99), dict(graph_rounds=-1), dict(walk_agg=2)):
        with pytest.raises(fora.FORAError) as ei:
            G1k.set_tuning(**bad)
        assert ei.value.code == fora.FORA_E_ARG
    assert G1k.get_tuning() == t


@pytest.mark.parametrize("shape", [dict(walk_blocks_per_cu=1, walk_chunk=64, push_blocks_per_cu=1),
                                   dict(walk_blocks_per_cu=16, walk_chunk=4096,
                                        push_blocks_per_cu=16),
                                   dict(walk_blocks_per_cu=4, walk_chunk=512, walk_agg=1)])
def test_results_do_not_depend_on_tuning(g1k, G1k, shape):
    ws0 = fora.workspace(G1k, 1)
    base = fora.fora_ssppr(G1k, 7, k=50, seed=3, ws=ws0, stats=True, flags=WC)
    v0 = _rows(G1k, 1, ws0)
    G1k.set_tuning(**shape)
    ws = fora.workspace(G1k, 1)
    res = fora.fora_ssppr(G1k, 7, k=50, seed=3, ws=ws, stats=True, flags=WC)
    v = _rows(G1k, 1, ws)
    _same_query(v, v0, 0, 0)
    assert torch.equal(res.ids, base.ids) and torch.equal(res.vals, base.vals)
    assert res.stats["steps"] == base.stats["steps"]
    exactcmp.check_query(g1k, G1k, 7, 0.2, res.stats["rmax"], exactcmp.row_of(
        fora.fora_workspace_views(G1k, 1, ws), 0), res.stats, key1=3)


def test_graph_replays_match_eager(g1k, G1k):
    srcs = [0, 3, 3, 500, 999, 42]
    qs = fora.make_queries(srcs, k=50, seed=[1, 2, 2, 3, 4, 5], n=g1k.n, flags=WC)
    B = len(srcs)
    ws_e = fora.workspace(G1k, B)
    eager = fora.fora_ssppr_batch(G1k, qs, ws=ws_e, stats=True)
    ref = _rows(G1k, B, ws_e)
    ref_ids = eager.ids.cpu().numpy()
    omega_unit = eager.stats[0]["omega_unit"]
    rounds = max(s["rounds"] for s in eager.stats)
    G1k.set_tuning(graph_rounds=rounds + 2)
    ws_g = fora.workspace(G1k, B)
    out = (torch.empty((B, 50), dtype=torch.int32, device="cuda"),
           torch.empty((B, 50), dtype=torch.float32, device="cuda"))
    for rep in range(3):
        res = fora.fora_ssppr_batch(G1k, qs, ws=ws_g, out=out, stats=True)
        torch.cuda.synchronize()
        got = _rows(G1k, B, ws_g)
        for b in range(B):
            _same_query(got, ref, b, b, omega_unit)
            order = np.lexsort((np.arange(g1k.n), -got["pi_hat"][b]))[:50]
            assert np.array_equal(res.ids[b].cpu().numpy(), order)
        assert [s["rounds"] for s in res.stats] == [s["rounds"] for s in eager.stats]
        # eager work on the same stream between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        fora.fora_ssppr(G1k, 11, k=5, seed=9)
    assert ref_ids.shape == (B, 50)


def test_graph_with_too_few_rounds_finishes_on_host(g1k, G1k):
    srcs = [0, 17]
    qs = fora.make_queries(srcs, k=50, seed=1, n=g1k.n, flags=WC)
    ws_e = fora.workspace(G1k, 2)
    eager = fora.fora_ssppr_batch(G1k, qs, ws=ws_e, stats=True)
    ref = _rows(G1k, 2, ws_e)
    G1k.set_tuning(graph_rounds=2)  # far fewer than the push needs
    ws_g = fora.workspace(G1k, 2)
    for _ in range(2):
        res = fora.fora_ssppr_batch(G1k, qs, ws=ws_g, stats=True)
        got = _rows(G1k, 2, ws_g)
        for b in range(2):
            _same_query(got, ref, b, b, eager.stats[0]["omega_unit"])
        assert [s["rounds"] for s in res.stats] == [s["rounds"] for s in eager.stats]


def test_shared_phase_memory_leaves_no_trace(g1k, G1k):
    # the push's frontier arrays and the walk phase's plan and sums share one
    # region of the workspace: a workspace filled with junk and then used by
    # push-only and walk-only calls gives the rows of a fresh one, and a
    # walk-only call with no plan entries leaves all-zero sums
    ws0 = fora.workspace(G1k, 1)
    base = fora.fora_ssppr(G1k, 7, k=50, seed=3, ws=ws0, stats=True, flags=WC)
    ref = _rows(G1k, 1, ws0)
    ws = fora.workspace(G1k, 1)
    ws.fill_(0xA5)
    fora.fora_push_only(G1k, 11, 0.2, 1e-6, ws=ws)
    w = fora.fora_walk_only(G1k, [], [], [], 1, 2, 0.2, ws=ws)
    assert w["steps"] == 0
    assert not w["cnt"].any().item() and not w["acc_fx"].any().item()
    fora.fora_push_only(G1k, 11, 0.2, 1e-6, ws=ws)
    res = fora.fora_ssppr(G1k, 7, k=50, seed=3, ws=ws, stats=True, flags=WC)
    _same_query(_rows(G1k, 1, ws), ref, 0, 0)
    assert torch.equal(res.ids, base.ids) and torch.equal(res.vals, base.vals)


def test_mixed_parameters_match_single_calls(g1k, G1k):
    srcs = [5, 5, 900, 64]
    eps = [0.5, 0.3, 0.5, 0.2]
    ks = [10, 50, 1, 200]
    alphas = [0.2, 0.2, 0.15, 0.3]
    qs = fora.make_queries(srcs, alpha=alphas, eps=eps, k=ks, seed=[0, 1, 2, 3], n=g1k.n,
                           flags=WC)
    B = len(srcs)
    ws = fora.workspace(G1k, B)
    bat = fora.fora_ssppr_batch(G1k, qs, kmax=200, ws=ws, stats=True)
    got = _rows(G1k, B, ws)
    ws1 = fora.workspace(G1k, 1)
    for b in range(B):
        single = fora.fora_ssppr(G1k, srcs[b], alphas[b], eps[b], k=ks[b], seed=b, ws=ws1,
                                 stats=True, flags=WC)
        one = _rows(G1k, 1, ws1)
        _same_query(got, one, b, 0, single.stats["omega_unit"])
        assert bat.stats[b]["omega_unit"] == single.stats["omega_unit"]
        assert bat.stats[b]["rmax"] == single.stats["rmax"]
        ids = bat.ids[b].cpu().numpy()
        assert np.all(ids[ks[b]:] == -1)
        ref = oracle.fora(g1k, srcs[b], alpha=alphas[b], eps=eps[b], k=ks[b], seed=b)
        assert bat.stats[b]["rounds"] == ref["rounds"]


def test_many_pulling_queries_match_single_calls(g1k, G1k):
    # 19 queries pull in the same rounds: groups of 8, 8 and 3 share each
    # chunk's in-edge scan; every row must equal its query run alone
    srcs = [int(x) for x in np.random.default_rng(5).integers(0, g1k.n, 19)]
    seeds = list(range(19))
    qs = fora.make_queries(srcs, k=50, seed=seeds, n=g1k.n, flags=WC)
    B = len(srcs)
    ws = fora.workspace(G1k, B)
    bat = fora.fora_ssppr_batch(G1k, qs, ws=ws, stats=True)
    got = _rows(G1k, B, ws)
    assert sum(s["pull_rounds"] for s in bat.stats) >= 3 * B
    ws1 = fora.workspace(G1k, 1)
    for b in range(B):
        single = fora.fora_ssppr(G1k, srcs[b], k=50, seed=seeds[b], ws=ws1, stats=True,
                                 flags=WC)
        one = _rows(G1k, 1, ws1)
        _same_query(got, one, b, 0, single.stats["omega_unit"])
        assert bat.stats[b]["rounds"] == single.stats["rounds"]
        assert bat.stats[b]["pull_rounds"] == single.stats["pull_rounds"]
    ref = oracle.fora(g1k, srcs[0], k=50, seed=seeds[0])
    assert bat.stats[0]["rounds"] == ref["rounds"]


def test_a_workspace_fits_every_smaller_batch(g1k, G1k):
    # the pull groups change with the batch (1, 4 or 16 queries), the
    # workspace size must not shrink with it: top-k FORA runs its later
    # iterations on the first one's workspace with fewer queries
    sizes = [fora.fora_workspace_size(G1k, b) for b in range(1, 41)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))
    ws = fora.workspace(G1k, 16)
    qs = fora.make_queries(list(range(15)), k=10, seed=1, n=g1k.n)
    res = fora.fora_ssppr_batch(G1k, qs, ws=ws, stats=True)
    assert all(s["walks"] > 0 for s in res.stats)


def test_maximum_batch(g1k, G1k):
    # FORA_MAX_BATCH queries in one call (256 pull groups of 16, the
    # per-query LDS staging at its largest); rows spot-checked against the
    # same queries run alone, and one query more is rejected
    B = fora.FORA_MAX_BATCH
    srcs = [int(x) for x in np.arange(B) % g1k.n]
    kw = dict(k=10, n=g1k.n, delta=1e-2, pf=1e-2)
    qs = fora.make_queries(srcs, seed=list(range(B)), **kw)
    res = fora.fora_ssppr_batch(G1k, qs, stats=True)
    assert all(s["walks"] > 0 and s["term_violations"] == 0 for s in res.stats)
    for b in (0, 1234, B - 1):
        one = fora.fora_ssppr(G1k, srcs[b], k=10, seed=b, delta=1e-2, pf=1e-2, stats=True)
        assert one.stats["rounds"] == res.stats[b]["rounds"]
        assert one.stats["omega_unit"] == res.stats[b]["omega_unit"]
        assert torch.equal(one.ids, res.ids[b]) and torch.equal(one.vals, res.vals[b])
        assert one.stats["steps"] == res.stats[b]["steps"]
    with pytest.raises(fora.FORAError) as ei:
        fora.fora_ssppr_batch(G1k, fora.make_queries(srcs + [0], seed=0, **kw))
    assert ei.value.code == fora.FORA_E_ARG


def test_autotune_sets_and_caches(g1k, G1k, tmp_path):
    qs = fora.make_queries([0, 1, 2, 3], k=50, n=g1k.n)
    path = str(tmp_path / "tune.json")
    rec = autotune.autotune(G1k, qs, path=path)
    assert not rec["cached"]
    t = G1k.get_tuning()
    assert t == rec["tuning"]
    rec2 = autotune.autotune(G1k, qs, path=path)
    assert rec2["cached"] and rec2["tuning"] == t
    res = fora.fora_ssppr_batch(G1k, qs, stats=True)
    ref = oracle.fora(g1k, 2, k=50, seed=0)
    assert res.stats[2]["rounds"] == ref["rounds"]
