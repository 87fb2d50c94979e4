"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (from the method's arithmetic):
* integer outputs (walk end-point counts, step totals, frontier sets, top-k
  ids of a given estimate) are bit-exact;
* residues (fixed point, 62 fraction bits) and FP32 reserves vs the FP64
  oracle replaying the device's own frontiers: every listed node passes the
  push test and no unlisted one fails it, within 1e-5 of its threshold, and
  |g - o| <= 1e-5 |o| + 1e-12 element by element; where the oracle's
  free-running push keeps every residue further than 1e-5 from its
  threshold, the frontiers themselves are equal;
* walk end-point counts and moves on the device's residues equal the
  oracle's walks on the plan of the same residues;
* walk weights: the GPU sums round(w * 2^62) per walk in integers, so it may
  differ from the FP64 sum by at most cnt * 2^-63 plus FP64 rounding;
* a query in a batch equals the same query alone bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.graphs import Graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora  # noqa: E402  (fails loudly if not built)
import exactcmp  # noqa: E402

ALPHA = 0.2
RTOL, ATOL = 1e-5, 1e-12


def close(g, o, rtol=RTOL, atol=ATOL):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return np.abs(g - o) <= rtol * np.abs(o) + atol


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def G1k(g1k):
    return fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)


@pytest.fixture(scope="module")
def grmat12():
    return synth.rmat_graph(12, seed=12, cache=False)


@pytest.fixture(scope="module")
def Grmat12(grmat12):
    return fora.Graph.from_numpy(grmat12.rowptr, grmat12.colidx)


def _cnt(t):
    """Walk end-point counts (uint64 bits in an int64 tensor) as numpy."""
    return t.cpu().numpy().view(np.uint64)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------ RNG
def test_philox_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(100003, 4), dtype=np.uint64).astype(np.uint32)
    for key in ([0, 0], [123, 456], [0xFFFFFFFF, 0x9E3779B9]):
        got = fora.fora_philox(ctr, key)
        want = oracle.philox(ctr, key)
        assert np.array_equal(got, want)


# ------------------------------------------------------------------ graph ingest
def test_build_csr_rejects_malformed():
    dev = "cuda"
    cases = [
        ([0, 1, 1], [1], fora.FORA_E_GRAPH),           # node 1 has no out-edge
        ([0, 1, 2], [1, 2], fora.FORA_E_GRAPH),        # target out of range
        ([0, 2, 1], [1], fora.FORA_E_GRAPH),           # rowptr decreasing / rowptr[n] != m
        ([1, 1, 2], [0, 1], fora.FORA_E_GRAPH),        # rowptr[0] != 0
    ]
    for rp, ci, code in cases:
        with pytest.raises(fora.FORAError) as ei:
            fora.Graph(torch.tensor(rp, dtype=torch.int32, device=dev),
                       torch.tensor(ci, dtype=torch.int32, device=dev))
        assert ei.value.code == code
    G = fora.Graph(torch.tensor([0, 1, 2], dtype=torch.int32, device=dev),
                   torch.tensor([1, 0], dtype=torch.int32, device=dev))
    assert G.max_degree == 1


@pytest.mark.parametrize("graph", ["rmat12", "hub", "uniform", "one"])
def test_degree_rank_is_a_stable_descending_sort(graph, grmat12):
    # the library's own radix sort against numpy's stable sort: out-degree
    # descending, equal degrees in id order (one, two and three byte passes)
    g = {"rmat12": grmat12, "hub": synth.hub_graph(70000, extra=1, seed=2),
         "uniform": synth.uniform_out_graph(1000, 10, seed=1),
         "one": Graph(np.array([0, 1], np.int32), np.array([0], np.int32))}[graph]
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    rank = fora.fora_graph_rank(G).cpu().numpy()
    order = np.argsort(-g.degrees(), kind="stable")
    want = np.empty(g.n, np.int64)
    want[order] = np.arange(g.n)
    assert np.array_equal(rank, want)
    G.close()


def test_argument_checks(G1k):
    ws = fora.workspace(G1k, 1)
    bad = [dict(src=-1), dict(src=1000), dict(alpha=0.0), dict(alpha=1.0), dict(eps=0.0),
           dict(eps=1.0), dict(delta=0.0), dict(pf=1.0), dict(k=0), dict(k=1001)]
    for b in bad:
        kw = dict(src=0, alpha=0.2, eps=0.5, delta=1e-3, pf=1e-3, k=50)
        kw.update(b)
        k = max(kw["k"], 1)
        with pytest.raises(fora.FORAError) as ei:
            fora.fora_ssppr(G1k, kw["src"], kw["alpha"], kw["eps"], kw["delta"], kw["pf"],
                            kw["k"], ws=ws,
                            out=(torch.empty(k, dtype=torch.int32, device="cuda"),
                                 torch.empty(k, dtype=torch.float32, device="cuda")))
        assert ei.value.code == fora.FORA_E_ARG
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(fora.FORAError) as ei:
        fora.fora_ssppr(G1k, 0, k=50, ws=small)
    assert ei.value.code == fora.FORA_E_NOMEM


def test_walk_index_overflow_is_an_error(G1k):
    # one push of the source leaves 0.08 on each of 10 neighbours; with
    # omega_unit ~ 7e10 each omega_v = ceil(0.08 omega_unit) >= 2^32 does not
    # fit the 32-bit walk index: the plan is rejected before any walk runs
    c = oracle.constants(10000, ALPHA, 0.5, 1e-9, 1e-3)
    assert 0.08 * c["omega_unit"] >= 2**32
    with pytest.raises(fora.FORAError) as ei:
        fora.fora_ssppr(G1k, 0, ALPHA, 0.5, 1e-9, 1e-3, 10, rmax=0.05)
    assert ei.value.code == fora.FORA_E_OVERFLOW
    # the library stays usable
    fora.fora_ssppr(G1k, 0, k=10)


# ------------------------------------------------------------------ push
def _push_compare(g, G, s, rmax):
    """The device's push against the oracle replaying its frontiers (always),
    and against the oracle's own free-running push (frontiers equal where no
    residue of that run comes within 1e-5 of its threshold)."""
    ref = oracle.push(g, s, ALPHA, rmax, log_frontiers=True)
    got = fora.fora_push_only(G, s, ALPHA, rmax, log_frontiers=True)
    exactcmp.check_push(g, s, ALPHA, rmax, got["frontiers"], got["r"].cpu().numpy(),
                        got["q"].cpu().numpy())
    if ref["min_margin"] > 1e-5:
        assert got["stats"]["rounds"] == ref["rounds"]
        assert np.array_equal(got["round_sizes"], ref["round_sizes"])
        for fg, fo in zip(got["frontiers"], ref["frontiers"]):
            assert np.array_equal(fg, fo)
    return ref, got


def test_push_golden_tiny():
    import json, os
    from conftest import GOLDEN
    gold = json.load(open(os.path.join(GOLDEN, "push_sync_tiny.json")))
    gr = gold["graph"]
    G = fora.Graph.from_numpy(np.array(gr["rowptr"]), np.array(gr["colidx"]))
    got = fora.fora_push_only(G, gold["source"], gold["alpha"], gold["rmax"], log_frontiers=True)
    assert got["stats"]["rounds"] == gold["rounds"]
    assert [list(f) for f in got["frontiers"]] == gold["frontiers"]
    assert np.all(close(got["q"].cpu().numpy(), gold["reserve"], rtol=1e-6))
    assert np.all(close(got["r"].cpu().numpy(), gold["residue"], rtol=1e-6))


@pytest.mark.parametrize("s", [0, 17, 999])
@pytest.mark.parametrize("rmax", [3.754e-5, 1e-3, 1e-6])
def test_push_parity_uniform(g1k, G1k, s, rmax):
    ref, got = _push_compare(g1k, G1k, s, rmax)
    # these cases keep every residue clear of its threshold: the free-running
    # comparison applies too
    assert ref["min_margin"] > 1e-5
    assert got["stats"]["rounds"] == ref["rounds"]
    assert np.array_equal(got["round_sizes"], ref["round_sizes"])
    for fg, fo in zip(got["frontiers"], ref["frontiers"]):
        assert np.array_equal(fg, fo)
    assert np.all(close(got["q"].cpu().numpy(), ref["q"]))
    assert np.all(close(got["r"].cpu().numpy(), ref["r"]))
    assert got["stats"]["edge_ops"] == ref["edge_ops"]
    assert got["stats"]["term_violations"] == 0


@pytest.mark.parametrize("pull_ratio", [0, 1 << 30])
@pytest.mark.parametrize("s", [0, 999])
def test_push_parity_forced_mode(g1k, s, pull_ratio):
    # pull_ratio 0: every round pushes; 2^30: every non-empty round pulls
    G = fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)
    G.set_tuning(pull_ratio=pull_ratio)
    ref, got = _push_compare(g1k, G, s, 3.754e-5)
    assert ref["min_margin"] > 1e-5
    if pull_ratio == 0:
        assert got["stats"]["pull_rounds"] == 0
    else:
        assert got["stats"]["pull_rounds"] == got["stats"]["rounds"]
    assert np.array_equal(got["round_sizes"], ref["round_sizes"])
    for fg, fo in zip(got["frontiers"], ref["frontiers"]):
        assert np.array_equal(fg, fo)
    assert np.all(close(got["q"].cpu().numpy(), ref["q"]))
    assert np.all(close(got["r"].cpu().numpy(), ref["r"]))


@pytest.mark.parametrize("pull_ratio", [0, 16, 1 << 30])
def test_push_parity_split_hubs(pull_ratio):
    # node 0 has out-degree n-1 and node 1 in-degree ~n-1: both are cut into
    # pieces (push: out-pieces; pull: in-pieces)
    g = synth.hub_graph(8000, seed=4)
    deg = g.degrees()
    indeg = np.bincount(g.colidx, minlength=g.n)
    assert deg[0] > 2048 and indeg[1] > 2048
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    G.set_tuning(pull_ratio=pull_ratio)
    # cases whose residues stay clear of their thresholds (the regular
    # structure puts many residues close to them at smaller r_max)
    for s, rmax in ((0, 6.812920690579608e-05), (5, 6.812920690579608e-05),
                    (77, 3.1622776601683795e-05)):
        ref, got = _push_compare(g, G, s, rmax)
        assert ref["min_margin"] > 1e-5
        assert np.array_equal(got["round_sizes"], ref["round_sizes"])
        for fg, fo in zip(got["frontiers"], ref["frontiers"]):
            assert np.array_equal(fg, fo)
        assert np.all(close(got["q"].cpu().numpy(), ref["q"]))
        assert np.all(close(got["r"].cpu().numpy(), ref["r"]))


@pytest.mark.parametrize("rmax", [1e-6, 1e-7])
def test_push_parity_rmat_ragged(grmat12, Grmat12, rmax):
    # every case through the replay; the free-running comparison where it applies
    deg = grmat12.degrees()
    for s in (int(np.argmax(deg)), 3, 4095):
        ref, got = _push_compare(grmat12, Grmat12, s, rmax)
        assert got["stats"]["term_violations"] == 0


# ------------------------------------------------------------------ walks
def _walk_compare(g, G, pv, po, pw, key0, key1):
    t_alpha = oracle.constants(g.m, ALPHA, 0.5, 0.01, 0.01)["t_alpha"]
    ref = oracle.walks(g, key0, key1, t_alpha, pv, po, pw)
    got = fora.fora_walk_only(G, pv, po, pw, key0, key1, ALPHA)
    cnt = _cnt(got["cnt"])
    assert np.array_equal(cnt, ref["cnt"])
    assert got["steps"] == ref["steps"]
    acc = _u64(got["acc_fx"]).astype(np.float64) / 2.0**62
    tol = ref["cnt"] * 2.0**-62 + 1e-15 * ref["acc"]
    assert np.all(np.abs(acc - ref["acc"]) <= tol)
    return ref, got


def test_walk_parity_oracle_plan(g1k, G1k):
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    ps = oracle.push(g1k, 0, ALPHA, c["rmax"])
    pv, po, pw = oracle.plan(ps["r"], c["omega_unit"])
    _walk_compare(g1k, G1k, pv, po, pw, 0, 7)


@pytest.mark.parametrize("seed", [0, 1])
def test_walk_parity_both_record_forms(grmat12, Grmat12, seed):
    # slots with the neighbour's id (the default where it fits, as here),
    # (start, degree) slots with the id read from the end node's header, and
    # ids with a 4-bit degree field (degrees of 15 or more from the header)
    pv, po, pw = synth.random_walk_plan(grmat12, 2000, 500, 40 + seed)
    t0 = Grmat12.get_tuning()
    assert t0["record_ids"] == 1
    try:
        for form in (0, 1, 2):
            Grmat12.set_tuning(record_ids=form)
            _walk_compare(grmat12, Grmat12, pv, po, pw, 5 + seed, 6)
    finally:
        Grmat12.set_tuning(**t0)
    with pytest.raises(fora.FORAError) as ei:
        Grmat12.set_tuning(record_ids=3)
    assert ei.value.code == fora.FORA_E_ARG


@pytest.mark.parametrize("entries,max_walks,seed", [(1, 1, 0), (1, 100000, 1), (7, 3, 2),
                                                    (4096, 1, 3), (3000, 300, 4),
                                                    (64, 513, 5), (1000, 2000, 6)])
def test_walk_parity_random_plans(grmat12, Grmat12, entries, max_walks, seed):
    pv, po, pw = synth.random_walk_plan(grmat12, entries, max_walks, seed)
    _walk_compare(grmat12, Grmat12, pv, po, pw, 11 + seed, 99)


@pytest.mark.parametrize("entries,max_walks,seed,chunk", [(1, 100000, 1, 64), (3000, 300, 4, 512),
                                                          (64, 513, 5, 4096), (4096, 1, 3, 256)])
def test_walk_parity_with_lds_aggregation(grmat12, Grmat12, entries, max_walks, seed, chunk):
    # end points summed in the waves' LDS tables first: counts and fixed-point
    # weights are integer sums, so they equal the direct path bit for bit
    pv, po, pw = synth.random_walk_plan(grmat12, entries, max_walks, seed)
    t0 = Grmat12.get_tuning()
    try:
        Grmat12.set_tuning(walk_agg=0, walk_chunk=chunk)
        direct = fora.fora_walk_only(Grmat12, pv, po, pw, 11 + seed, 99, ALPHA)
        d_cnt, d_acc = _cnt(direct["cnt"]).copy(), _u64(direct["acc_fx"]).copy()
        Grmat12.set_tuning(walk_agg=1, walk_chunk=chunk)
        _, got = _walk_compare(grmat12, Grmat12, pv, po, pw, 11 + seed, 99)
        assert np.array_equal(_cnt(got["cnt"]), d_cnt)
        assert np.array_equal(_u64(got["acc_fx"]), d_acc)
        assert got["steps"] == direct["steps"]
    finally:
        Grmat12.set_tuning(**t0)


@pytest.mark.parametrize("bad_v", [[0, 1000], [-1, 3], [5, 5], [7, 3]])
def test_walk_only_rejects_bad_plans_on_the_device(G1k, bad_v):
    # node ids outside [0, n) or not strictly increasing: rejected before any
    # walk reads the node table
    v = np.array(bad_v, np.int32)
    with pytest.raises(fora.FORAError) as ei:
        fora.fora_walk_only(G1k, v, np.ones(2, np.uint64), np.full(2, 0.5), 0, 0, ALPHA)
    assert ei.value.code == fora.FORA_E_ARG
    # and the next good call works
    got = fora.fora_walk_only(G1k, np.array([0, 1], np.int32), np.ones(2, np.uint64),
                              np.full(2, 0.5), 0, 0, ALPHA)
    assert int(_cnt(got["cnt"]).sum()) == 2


def test_walk_only_empty_plan(G1k):
    got = fora.fora_walk_only(G1k, np.zeros(0, np.int32), np.zeros(0, np.uint64),
                              np.zeros(0), 0, 0, ALPHA)
    assert got["steps"] == 0
    assert int(_cnt(got["cnt"]).sum()) == 0


# ------------------------------------------------------------------ end to end
def _e2e(g, G, s, k, seed, rmax=None, eps=0.5):
    ref = oracle.fora(g, s, alpha=ALPHA, eps=eps, k=k, seed=seed, rmax=rmax)
    ws = fora.workspace(G, 1)
    res = fora.fora_ssppr(G, s, alpha=ALPHA, eps=eps, k=k, seed=seed, rmax=rmax, ws=ws,
                          stats=True, flags=fora.FORA_WALK_COUNTS)
    return ref, res, fora.fora_workspace_views(G, 1, ws)


def _estimate_is_reserve_plus_walks(row):
    # pi_hat = q + (walk weights), formed in FP64 and rounded once to FP32
    acc = row["walk_weight_fx"].view(np.uint64).astype(np.float64) * 2.0**-62
    want = (row["reserve"].astype(np.float64) + acc).astype(np.float32)
    assert np.array_equal(row["pi_hat"], want)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_end_to_end_uniform(g1k, G1k, seed):
    ref, res, v = _e2e(g1k, G1k, 0, 50, seed)
    st = res.stats
    assert 0 < st["pull_rounds"] < st["rounds"]  # both round kinds are exercised
    assert st["omega_unit"] == ref["consts"]["omega_unit"]
    assert st["rmax"] == ref["consts"]["rmax"]
    assert st["t_alpha"] == ref["consts"]["t_alpha"]
    assert st["rounds"] == ref["rounds"] and st["term_violations"] == 0
    row = exactcmp.row_of(v, 0)
    # push against the replay of its frontiers, walks against the oracle's
    # walks on the device's own residues: element by element, counts exact
    exactcmp.check_query(g1k, G1k, 0, ALPHA, st["rmax"], row, st, key1=seed)
    # the free-running oracle agrees as well (no residue sits within 1e-5 of
    # its threshold here): same plan, hence the same walks
    assert ref["min_margin"] > 1e-5
    assert np.all(close(row["reserve"], ref["q"])) and np.all(close(row["residue"], ref["r"]))
    assert st["walks"] == ref["walks"] and st["steps"] == ref["steps"]
    assert np.array_equal(_cnt(v["walk_count"][0]), ref["cnt"])
    _estimate_is_reserve_plus_walks(row)
    pi = row["pi_hat"]
    assert abs(pi.astype(np.float64).sum() - 1.0) < 1e-4
    ids = res.ids.cpu().numpy()
    vals = res.vals.cpu().numpy()
    # top-k of the GPU's own estimate is exact (a sort decides it)
    order = np.lexsort((np.arange(g1k.n), -pi))[:50]
    assert np.array_equal(ids, order)
    assert np.array_equal(vals, pi[order])
    # against the oracle: differences only between near-ties
    kth = ref["topk_vals"][-1]
    diff = set(ids.tolist()) ^ set(ref["topk_ids"].tolist())
    for t in diff:
        assert abs(ref["pi"][t] - kth) <= 2e-5 * kth + 1e-9


@pytest.mark.parametrize("agg", [0, 1])
def test_walk_counts_flag_changes_only_the_counts(g1k, G1k, agg):
    # the single-query entry point (no counts) against a batch of one that
    # asks for them: every other output is bit-identical (the push is
    # order-independent, so the two runs push identically)
    t0 = G1k.get_tuning()
    G1k.set_tuning(walk_agg=agg)
    try:
        ws_a, ws_b = fora.workspace(G1k, 1), fora.workspace(G1k, 1)
        a = fora.fora_ssppr(G1k, 3, alpha=ALPHA, k=50, seed=8, ws=ws_a, stats=True)
        b = fora.fora_ssppr(G1k, 3, alpha=ALPHA, k=50, seed=8, ws=ws_b, stats=True,
                            flags=fora.FORA_WALK_COUNTS)
        va = {k: t[0].cpu().numpy() for k, t in fora.fora_workspace_views(G1k, 1, ws_a).items()}
        vb = {k: t[0].cpu().numpy() for k, t in fora.fora_workspace_views(G1k, 1, ws_b).items()}
        assert not va["walk_count"].any()
        assert int(vb["walk_count"].view(np.uint64).sum()) == b.stats["walks"] > 0
        for key in ("residue_fx", "reserve", "walk_weight_fx", "pi_hat"):
            assert np.array_equal(va[key], vb[key]), key
        assert torch.equal(a.ids, b.ids) and torch.equal(a.vals, b.vals)
        for key in ("rounds", "walks", "steps", "omega_unit", "rmax"):
            assert a.stats[key] == b.stats[key], key
    finally:
        G1k.set_tuning(**t0)


def test_end_to_end_monte_carlo_case(g1k, G1k):
    ref, res, v = _e2e(g1k, G1k, 0, 50, 5, rmax=1.0)
    assert res.stats["rounds"] == 0 and ref["rounds"] == 0
    assert res.stats["walks"] == ref["walks"] == math.ceil(ref["consts"]["omega_unit"])
    assert res.stats["steps"] == ref["steps"]
    assert np.array_equal(_cnt(v["walk_count"][0]), ref["cnt"])


@pytest.mark.parametrize("k", [1, 7, 500, 1000])
def test_topk_sizes(g1k, G1k, k):
    res = fora.fora_ssppr(G1k, 3, k=k, seed=9, delta=1e-3, pf=1e-3)
    ws_pi = None
    ids = res.ids.cpu().numpy()
    assert len(set(ids.tolist())) == k
    vals = res.vals.cpu().numpy()
    assert np.all(np.diff(vals) <= 0)
    del ws_pi


def test_tiny_graph_self_loop_and_full_k():
    # n = 1 with a self-loop; and a 2-node cycle with k = n (padding rules)
    G = fora.Graph.from_numpy(np.array([0, 1]), np.array([0]))
    res = fora.fora_ssppr(G, 0, k=1, seed=0, delta=0.5, pf=0.5)
    assert res.ids.cpu().tolist() == [0]
    assert abs(float(res.vals.cpu()[0]) - 1.0) < 1e-6
    G2 = fora.Graph.from_numpy(np.array([0, 1, 2]), np.array([1, 0]))
    res = fora.fora_ssppr(G2, 1, k=2, seed=0, delta=0.5, pf=0.5)
    assert sorted(res.ids.cpu().tolist()) == [0, 1]


# ------------------------------------------------------------------ batch
def test_batch_matches_single(g1k, G1k):
    srcs = [0, 5, 5, 999, 123]
    seeds = [1, 2, 2, 3, 4]
    qs = fora.make_queries(srcs, k=50, seed=seeds, n=g1k.n, flags=fora.FORA_WALK_COUNTS)
    ws = fora.workspace(G1k, len(srcs))
    out = fora.fora_ssppr_batch(G1k, qs, ws=ws, stats=True)
    vb = fora.fora_workspace_views(G1k, len(srcs), ws)
    ws1 = fora.workspace(G1k, 1)
    for i, (s, sd) in enumerate(zip(srcs, seeds)):
        row = exactcmp.row_of(vb, i)
        st = out.stats[i]
        # the same query alone: bit for bit
        one = fora.fora_ssppr(G1k, s, k=50, seed=sd, ws=ws1, stats=True,
                              flags=fora.FORA_WALK_COUNTS)
        alone = exactcmp.row_of(fora.fora_workspace_views(G1k, 1, ws1), 0)
        for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
            assert np.array_equal(row[key], alone[key]), key
        assert torch.equal(one.ids, out.ids[i]) and torch.equal(one.vals, out.vals[i])
        for key in ("rounds", "pushes", "edge_ops", "walks", "steps", "r_sum"):
            assert one.stats[key] == st[key], key
        # against the oracle, element by element
        exactcmp.check_query(g1k, G1k, s, ALPHA, st["rmax"], row, st, key1=sd)
        _estimate_is_reserve_plus_walks(row)
        order = np.lexsort((np.arange(g1k.n), -row["pi_hat"]))[:50]
        assert np.array_equal(out.ids[i].cpu().numpy(), order)
    # duplicates (same source and seed) are identical
    for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
        assert torch.equal(vb[key][1], vb[key][2]), key


def test_batch_of_mixed_queries_equals_each_alone(grmat12, Grmat12):
    # different eps, k, r_max and seeds share the batch's launches (pull
    # groups of 16, one walk launch): each row equals its query alone
    rng = np.random.default_rng(5)
    B = 24
    srcs = rng.integers(0, grmat12.n, B)
    srcs[3] = srcs[4]
    eps = rng.choice([0.1, 0.3, 0.5], B)
    ks = rng.choice([1, 50, 500], B)
    rmaxes = np.where(rng.random(B) < 0.3, 1e-6, 0.0)
    seeds = rng.integers(0, 2**31, B)
    qs = fora.make_queries(srcs, eps=eps, k=ks, rmax=rmaxes, seed=seeds, n=grmat12.n,
                           flags=fora.FORA_WALK_COUNTS)
    ws = fora.workspace(Grmat12, B)
    out = fora.fora_ssppr_batch(Grmat12, qs, kmax=500, ws=ws, stats=True)
    vb = fora.fora_workspace_views(Grmat12, B, ws)
    ws1 = fora.workspace(Grmat12, 1)
    for i in range(B):
        one = fora.fora_ssppr(Grmat12, int(srcs[i]), eps=float(eps[i]), k=int(ks[i]),
                              rmax=float(rmaxes[i]) or None, seed=int(seeds[i]), ws=ws1,
                              stats=True, flags=fora.FORA_WALK_COUNTS)
        alone = exactcmp.row_of(fora.fora_workspace_views(Grmat12, 1, ws1), 0)
        row = exactcmp.row_of(vb, i)
        for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
            assert np.array_equal(row[key], alone[key]), (i, key)
        k = int(ks[i])
        assert torch.equal(one.ids, out.ids[i, :k]) and torch.equal(one.vals, out.vals[i, :k])
    # and every row against the oracle
    for i in (0, 3, 7, 23):
        exactcmp.check_query(grmat12, Grmat12, int(srcs[i]), ALPHA, out.stats[i]["rmax"],
                             exactcmp.row_of(vb, i), out.stats[i], key1=int(seeds[i]))
